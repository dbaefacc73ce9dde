"""The C ABI library builds, loads and exports every entry point include/ncorp.h
declares; host-side argument checks work without a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nc():
    from paper_2310_20374_amd import ncorp
    if not os.path.exists(ncorp.LIB_PATH):
        from paper_2310_20374_amd import build
        build.build()
    return ncorp


def _declared():
    h = open(os.path.join(ROOT, "include", "ncorp.h")).read()
    return sorted(set(re.findall(r"\b(ncorp_[a-z_]+)\s*\(", h)))


def test_header_symbols_exported(nc):
    L = nc.lib()
    names = _declared()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert set(nc.EXPORTED_SYMBOLS) <= set(names)


def test_params_default_and_validation(nc):
    L = nc.lib()
    for p in range(7):
        prm = nc.params_default(p)
        assert prm.p == p
        assert prm.leaf_size == (17 if p <= 3 else 52)
        assert (prm.ncs_col, prm.ncc_pre_col, prm.ncc_post_col) == (12, 0, 16)
        assert (prm.collision_mode, prm.collision_f) == (nc.COLLISIONS_REPORT, 2.0)
        assert (prm.gravity_method, prm.ncb_pre, prm.ncb_post) == (nc.GRAVITY_FALCON, 6, 16)
        assert (prm.collision_method, prm.mesh_cells, prm.mesh_neighbours,
                prm.mesh_aspect, prm.mesh_gamma) == (nc.COLLISIONS_TREE, 256, 8.0, 0.05, 0.0)
        assert (prm.p2p_tile, prm.p2p_targets_max, prm.walk_waves) == (0, 0, 0)
    bad = nc.Params()
    assert L.ncorp_params_default(C.byref(bad), 7) == nc.E_INVALID
    h = C.c_void_p()
    for field, val in (("p", 7), ("theta_min", 1.0), ("theta_min", 0.0), ("leaf_size", 0),
                       ("ncs", -1), ("theta_mode", 2), ("precision", 5),
                       ("root_half_width", 3.0), ("G", -1.0), ("collision_mode", 2),
                       ("collision_f", 0.9), ("collision_f", 2.1), ("M_sun", -1.0),
                       ("obliquity", float("nan")), ("gravity_method", 4), ("ncb_pre", -1),
                       ("ncb_post", -1), ("collision_method", 4), ("mesh_cells", 0),
                       ("mesh_cells", -3), ("mesh_neighbours", 0.0), ("mesh_gamma", -1.0),
                       ("mesh_aspect", float("inf")), ("mesh_rmax", -1.0),
                       ("p2p_tile", 64), ("p2p_tile", 300), ("p2p_targets_max", 5),
                       ("p2p_targets_max", -1), ("walk_waves", 128), ("walk_waves", 4096)):
        prm = nc.params_default(3)
        setattr(prm, field, val)
        assert L.ncorp_create(C.byref(prm), C.byref(h)) == nc.E_INVALID, field
    prm = nc.params_default(3, J2=1e-3, R_central=0.0)       # J2 needs a radius
    assert L.ncorp_create(C.byref(prm), C.byref(h)) == nc.E_INVALID
    prm = nc.params_default(3, M_sun=1.0, a_sun=0.0)         # a distant body needs its orbit
    assert L.ncorp_create(C.byref(prm), C.byref(h)) == nc.E_INVALID
    prm = nc.params_default(3, root_half_width=16.0)
    assert L.ncorp_create(C.byref(prm), C.byref(h)) == nc.OK
    assert h.value
    # calls that need a tree or arrays fail on the host, before any GPU work
    assert L.ncorp_gravity(h, None, None, None, None, None) == nc.E_INVALID
    assert b"tree" in L.ncorp_last_error(h)
    assert L.ncorp_build_tree(h, None, None, None, 10, None, 0, None) == nc.E_INVALID
    L.ncorp_destroy(h)


def test_workspace_bytes(nc):
    prm = nc.params_default(6)
    a = nc.workspace_bytes(prm, 1000)
    b = nc.workspace_bytes(prm, 10 ** 6)
    assert 0 < a < b
    assert b % 256 == 0
    assert nc.workspace_bytes(prm, 1000, 10 ** 6) > a
    assert nc.lib().ncorp_workspace_bytes(C.byref(prm), 0, 0) == -1


def test_batched_argument_checks(nc):
    """The batched entry points reject a missing offset array and a disk count
    outside 1..NCORP_MAX_DISKS on the host, before any GPU work."""
    L = nc.lib()
    h = C.c_void_p()
    prm = nc.params_default(3)
    assert L.ncorp_create(C.byref(prm), C.byref(h)) == nc.OK
    dummy = C.c_void_p(256)          # never dereferenced: the checks come first
    assert L.ncorp_build_tree_batched(h, None, 4, dummy, dummy, dummy, 10, None, 0,
                                      None) == nc.E_INVALID
    assert b"disk_offsets" in L.ncorp_last_error(h)
    for nd in (0, -3, nc.MAX_DISKS + 1):
        assert L.ncorp_build_tree_batched(h, dummy, nd, dummy, dummy, dummy, 10, None, 0,
                                          None) == nc.E_INVALID
        assert b"n_disks" in L.ncorp_last_error(h)
        assert L.ncorp_step_batched(h, dummy, nd, *([dummy] * 8), 10, 1e-3, 1, None, 0, dummy,
                                    None, 0, None) == nc.E_INVALID
    # a valid disk count still needs positions and a workspace
    assert L.ncorp_build_tree_batched(h, dummy, 2, None, None, None, 10, None, 0,
                                      None) == nc.E_INVALID
    assert L.ncorp_build_tree_batched(h, dummy, 2, dummy, dummy, dummy, 10, None, 0,
                                      None) == nc.E_INVALID
    assert b"workspace" in L.ncorp_last_error(h)
    L.ncorp_destroy(h)


def test_noalloc_rejects_sizes_beyond_its_array(nc):
    """The allocation-free step refuses an n whose workspace would not fit its fixed
    per-GPU array, and bad arguments, on the host before any GPU work."""
    L = nc.lib()
    h = C.c_void_p()
    prm = nc.params_default(6)
    assert L.ncorp_create(C.byref(prm), C.byref(h)) == nc.OK
    dummy = C.c_void_p(256)          # never dereferenced: the checks come first
    limit = nc.STATIC_WORKSPACE_BYTES
    n_small = 2000
    assert nc.workspace_bytes(prm, n_small, 1) <= limit
    n_big = 10 ** 6
    assert nc.workspace_bytes(prm, n_big, 1) > limit
    args = [dummy] * 8
    assert L.ncorp_step_noalloc(h, *args, n_big, 1e-3, 1, dummy, 16, dummy, None) == nc.E_INVALID
    assert b"allocation-free" in L.ncorp_last_error(h)
    assert L.ncorp_step_noalloc(h, *args, 0, 1e-3, 1, dummy, 16, dummy, None) == nc.E_INVALID
    assert L.ncorp_step_noalloc(h, *args, n_small, 0.0, 1, dummy, 16, dummy, None) == nc.E_INVALID
    assert L.ncorp_step_noalloc(h, *args, n_small, 1e-3, 0, dummy, 16, dummy, None) == nc.E_INVALID
    assert L.ncorp_step_noalloc(h, None, *args[1:], n_small, 1e-3, 1, dummy, 16, dummy,
                                None) == nc.E_INVALID
    L.ncorp_destroy(h)


def test_autotune_cache_key():
    from paper_2310_20374_amd import autotune
    assert autotune.cache_key(4, 1, 788736) == "p4-prec1-n2^19"
    assert autotune.cache_key(6, 0, 1) == "p6-prec0-n2^0"
    assert autotune.CANDIDATES == tuple(sorted(autotune.CANDIDATES))

"""ctypes binding of libncorp (include/ncorp.h).  Argument marshalling only: every
step of the tree step runs in the library's HIP kernels.  torch tensors provide
device memory and the stream; nothing here computes.

The library must have been built (``paper_2310_20374_amd/build.py``); importing
this module on a machine without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libncorp.so")

OK, E_INVALID, E_CAPACITY, E_HIP, E_UNSUPPORTED, E_NONFINITE = 0, -1, -2, -3, -4, -5
FP64, FP32_BULK = 0, 1
COLLISIONS_REPORT, COLLISIONS_RESOLVE = 0, 1
GRAVITY_FALCON, GRAVITY_STANDARD_TREE, GRAVITY_MESH, GRAVITY_BRUTE_FORCE = 0, 1, 2, 3
COLLISIONS_TREE, COLLISIONS_MESH, COLLISIONS_STANDARD_TREE, COLLISIONS_BRUTE_FORCE = 0, 1, 2, 3
STATUS_NAMES = {0: "ok", -1: "invalid", -2: "capacity", -3: "hip", -4: "unsupported",
                -5: "nonfinite"}

INFO_FIELDS = ("n", "ncells", "nleaves", "maxlevel", "m2l", "p2p", "visited", "col_cand",
               "col_tests", "m2l_dir", "p2p_inter", "m2l_maxlist", "p2p_maxlist", "nroots",
               "long_m2l", "long_p2p", "walk_busy_max", "walk_busy_mean", "p2p_src_max",
               "sort_prev", "sort_spill")
PHASES = ("keys", "sort", "tree", "gclimb", "gwalk", "m2l", "descent", "p2p", "l2p", "collide",
          "integrate")
EXPORT = {"keys": 0, "perm": 1, "cells": 2, "gcells": 3, "ccells": 4, "multipoles": 5,
          "local": 6, "m2l": 7, "p2p": 8, "col_cand": 9}

EXPORTED_SYMBOLS = ("ncorp_params_default", "ncorp_create", "ncorp_destroy",
                    "ncorp_workspace_bytes", "ncorp_build_tree", "ncorp_gravity",
                    "ncorp_collide", "ncorp_step", "ncorp_get_status", "ncorp_last_error",
                    "ncorp_tree_info", "ncorp_export_host", "ncorp_set_timing",
                    "ncorp_phase_times", "ncorp_build_tree_batched", "ncorp_step_batched",
                    "ncorp_build_mesh", "ncorp_mesh_state", "ncorp_step_noalloc")
MAX_DISKS = 65536
STATIC_WORKSPACE_BYTES = 128 * 1024 * 1024     # NCORP_STATIC_WORKSPACE_BYTES


class Params(C.Structure):
    _fields_ = [
        ("G", C.c_double), ("M_central", C.c_double), ("p", C.c_int),
        ("theta_min", C.c_double), ("theta_mode", C.c_int), ("leaf_size", C.c_int),
        ("ncs", C.c_int), ("ncc_pre", C.c_int), ("ncc_post", C.c_int),
        ("ncs_col", C.c_int), ("ncc_pre_col", C.c_int), ("ncc_post_col", C.c_int),
        ("precision", C.c_int), ("root_half_width", C.c_double),
        ("cell_capacity", C.c_int64), ("m2l_capacity", C.c_int64),
        ("p2p_capacity", C.c_int64), ("queue_capacity", C.c_int64),
        ("m2l_per_cell", C.c_int32), ("p2p_per_leaf", C.c_int32),
        ("collision_mode", C.c_int32), ("collision_f", C.c_double),
        ("J2", C.c_double), ("R_central", C.c_double), ("M_sun", C.c_double),
        ("a_sun", C.c_double), ("obliquity", C.c_double), ("t_start", C.c_double),
        ("gravity_method", C.c_int32), ("ncb_pre", C.c_int32), ("ncb_post", C.c_int32),
        ("collision_method", C.c_int32), ("mesh_cells", C.c_int32),
        ("mesh_neighbours", C.c_double), ("mesh_aspect", C.c_double),
        ("mesh_rmax", C.c_double), ("mesh_min_side", C.c_double), ("mesh_gamma", C.c_double),
        ("p2p_tile", C.c_int32), ("p2p_targets_max", C.c_int32), ("walk_waves", C.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NcorpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ncorp error {code} ({STATUS_NAMES.get(code, '?')}): {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libncorp.so not built ({LIB_PATH}); run paper_2310_20374_amd/build.py")
    # torch brings its own HIP runtime (same soname as the system one); load it
    # first so libncorp binds to that single runtime instead of a second copy
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    vp, i64, i32, d = C.c_void_p, C.c_int64, C.c_int, C.c_double
    P = C.POINTER(Params)
    L.ncorp_params_default.argtypes = [P, i32]
    L.ncorp_params_default.restype = i32
    L.ncorp_create.argtypes = [P, C.POINTER(vp)]
    L.ncorp_create.restype = i32
    L.ncorp_destroy.argtypes = [vp]
    L.ncorp_destroy.restype = None
    L.ncorp_workspace_bytes.argtypes = [P, i64, i64]
    L.ncorp_workspace_bytes.restype = i64
    L.ncorp_build_tree.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp]
    L.ncorp_build_tree.restype = i32
    L.ncorp_build_mesh.argtypes = [vp, vp, vp, vp, vp, i64, vp, i64, vp]
    L.ncorp_build_mesh.restype = i32
    L.ncorp_mesh_state.argtypes = [vp, C.POINTER(C.c_double)]
    L.ncorp_mesh_state.restype = i32
    L.ncorp_gravity.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ncorp_gravity.restype = i32
    L.ncorp_collide.argtypes = [vp, vp, vp, vp, vp, d, vp, i64, vp, vp]
    L.ncorp_collide.restype = i32
    L.ncorp_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, d, i32, vp, i64, vp, vp,
                             i64, vp]
    L.ncorp_step.restype = i32
    L.ncorp_step_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, d, i32, vp, i64,
                                     vp, vp]
    L.ncorp_step_noalloc.restype = i32
    L.ncorp_build_tree_batched.argtypes = [vp, vp, i32, vp, vp, vp, i64, vp, i64, vp]
    L.ncorp_build_tree_batched.restype = i32
    L.ncorp_step_batched.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, i64, d, i32,
                                     vp, i64, vp, vp, i64, vp]
    L.ncorp_step_batched.restype = i32
    L.ncorp_get_status.argtypes = [vp, C.POINTER(i64)]
    L.ncorp_get_status.restype = i32
    L.ncorp_last_error.argtypes = [vp]
    L.ncorp_last_error.restype = C.c_char_p
    L.ncorp_tree_info.argtypes = [vp, C.POINTER(i64)]
    L.ncorp_tree_info.restype = i32
    L.ncorp_export_host.argtypes = [vp, i32, vp, i64]
    L.ncorp_export_host.restype = i64
    L.ncorp_set_timing.argtypes = [vp, i32]
    L.ncorp_set_timing.restype = i32
    L.ncorp_phase_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
    L.ncorp_phase_times.restype = i32
    _lib = L
    return L


def params_default(p: int = 3, **over) -> Params:
    prm = Params()
    r = lib().ncorp_params_default(C.byref(prm), int(p))
    if r != OK:
        raise NcorpError(r, "ncorp_params_default")
    for k, v in over.items():
        if not hasattr(prm, k):
            raise KeyError(k)
        setattr(prm, k, v)
    return prm


def workspace_bytes(prm: Params, n_max: int, pair_capacity: int = 1 << 16) -> int:
    b = lib().ncorp_workspace_bytes(C.byref(prm), int(n_max), int(pair_capacity))
    if b < 0:
        raise NcorpError(E_INVALID, "ncorp_workspace_bytes rejected its arguments")
    return int(b)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """One ncorp_ctx plus its (caller-owned) device workspace."""

    def __init__(self, prm: Params, n_max: int, pair_capacity: int = 1 << 16,
                 device: str = "cuda:0"):
        """n_max = 0: no workspace (only ncorp_step_noalloc can then be called)."""
        import torch
        self.prm = prm
        self.h = C.c_void_p()
        r = lib().ncorp_create(C.byref(prm), C.byref(self.h))
        if r != OK:
            raise NcorpError(r, "ncorp_create rejected the parameters")
        self.device = device
        if n_max == 0:
            self._raw, self.ws, self.ws_bytes = None, None, 0
            return
        self.ws_bytes = workspace_bytes(prm, n_max, pair_capacity)
        raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[off: off + self.ws_bytes]
        self.device = device

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().ncorp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, r, what):
        if r != OK:
            raise NcorpError(r, f"{what}: {lib().ncorp_last_error(self.h).decode()}")

    # ---- entry points (same names as the C ABI)
    def build_tree(self, x, y, z, stream=None):
        n = x.numel()
        self._check(lib().ncorp_build_tree(self.h, _ptr(x), _ptr(y), _ptr(z), n,
                                           _ptr(self.ws), self.ws_bytes, _stream(stream)),
                    "ncorp_build_tree")

    def build_mesh(self, x, y, z, R, stream=None):
        n = x.numel()
        self._check(lib().ncorp_build_mesh(self.h, _ptr(x), _ptr(y), _ptr(z), _ptr(R), n,
                                           _ptr(self.ws), self.ws_bytes, _stream(stream)),
                    "ncorp_build_mesh")

    def mesh_state(self):
        """(gamma, measured mean neighbours x' or nan, moonlets in the mesh, out of it)."""
        out = (C.c_double * 4)()
        self._check(lib().ncorp_mesh_state(self.h, out), "ncorp_mesh_state")
        return {"gamma": out[0], "neighbours": out[1], "n_in": int(out[2]),
                "n_out": int(out[3])}

    def gravity(self, m, ax, ay, az, stream=None):
        self._check(lib().ncorp_gravity(self.h, _ptr(m), _ptr(ax), _ptr(ay), _ptr(az),
                                        _stream(stream)), "ncorp_gravity")

    def collide(self, vx, vy, vz, R, dt, pairs, n_pairs_dev, stream=None):
        cap = pairs.shape[0] if pairs is not None else 0
        self._check(lib().ncorp_collide(self.h, _ptr(vx), _ptr(vy), _ptr(vz), _ptr(R),
                                        float(dt), _ptr(pairs), cap, _ptr(n_pairs_dev),
                                        _stream(stream)), "ncorp_collide")

    def step(self, x, y, z, vx, vy, vz, m, R, dt, n_steps, pairs, n_pairs_dev, stream=None):
        cap = pairs.shape[0] if pairs is not None else 0
        self._check(lib().ncorp_step(self.h, _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy),
                                     _ptr(vz), _ptr(m), _ptr(R), x.numel(), float(dt),
                                     int(n_steps), _ptr(pairs), cap, _ptr(n_pairs_dev),
                                     _ptr(self.ws), self.ws_bytes, _stream(stream)),
                    "ncorp_step")

    def step_noalloc(self, x, y, z, vx, vy, vz, m, R, dt, n_steps, pairs, n_pairs_dev,
                     stream=None):
        """ncorp_step on the library's fixed per-GPU workspace (no workspace argument)."""
        cap = pairs.shape[0] if pairs is not None else 0
        self._check(lib().ncorp_step_noalloc(self.h, _ptr(x), _ptr(y), _ptr(z), _ptr(vx),
                                             _ptr(vy), _ptr(vz), _ptr(m), _ptr(R), x.numel(),
                                             float(dt), int(n_steps), _ptr(pairs), cap,
                                             _ptr(n_pairs_dev), _stream(stream)),
                    "ncorp_step_noalloc")

    def build_tree_batched(self, offsets, x, y, z, stream=None):
        """offsets: int64 device tensor of n_disks + 1 entries."""
        self._check(lib().ncorp_build_tree_batched(self.h, _ptr(offsets), offsets.numel() - 1,
                                                   _ptr(x), _ptr(y), _ptr(z), x.numel(),
                                                   _ptr(self.ws), self.ws_bytes,
                                                   _stream(stream)),
                    "ncorp_build_tree_batched")

    def step_batched(self, offsets, x, y, z, vx, vy, vz, m, R, dt, n_steps, pairs, n_pairs_dev,
                     stream=None):
        cap = pairs.shape[0] if pairs is not None else 0
        self._check(lib().ncorp_step_batched(self.h, _ptr(offsets), offsets.numel() - 1,
                                             _ptr(x), _ptr(y), _ptr(z), _ptr(vx), _ptr(vy),
                                             _ptr(vz), _ptr(m), _ptr(R), x.numel(), float(dt),
                                             int(n_steps), _ptr(pairs), cap, _ptr(n_pairs_dev),
                                             _ptr(self.ws), self.ws_bytes, _stream(stream)),
                    "ncorp_step_batched")

    def get_status(self):
        req = C.c_int64(0)
        r = lib().ncorp_get_status(self.h, C.byref(req))
        return r, int(req.value), lib().ncorp_last_error(self.h).decode()

    def check_status(self):
        r, req, msg = self.get_status()
        if r != OK:
            raise NcorpError(r, f"{msg} (required {req})")

    def set_timing(self, enable: bool = True):
        self._check(lib().ncorp_set_timing(self.h, 1 if enable else 0), "ncorp_set_timing")

    def phase_times(self):
        """{phase: (milliseconds, launches)} accumulated since the last call."""
        ms = (C.c_double * len(PHASES))()
        cnt = (C.c_int64 * len(PHASES))()
        self._check(lib().ncorp_phase_times(self.h, ms, cnt), "ncorp_phase_times")
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(PHASES)}

    def tree_info(self):
        arr = (C.c_int64 * len(INFO_FIELDS))()
        self._check(lib().ncorp_tree_info(self.h, arr), "ncorp_tree_info")
        return dict(zip(INFO_FIELDS, [int(v) for v in arr]))

    def export(self, what: str):
        """Copy an internal array to host (numpy), for tests and tuning."""
        import numpy as np
        code = EXPORT[what]
        need = lib().ncorp_export_host(self.h, code, None, 0)
        if need < 0:
            self._check(int(need), f"export {what}")
        buf = np.empty(max(int(need), 1), dtype=np.uint8)
        got = lib().ncorp_export_host(self.h, code, buf.ctypes.data_as(C.c_void_p), int(need))
        if got < 0:
            self._check(int(got), f"export {what}")
        buf = buf[: int(need)]
        if what == "keys":
            return buf.view(np.uint64)
        if what == "perm":
            return buf.view(np.uint32)
        if what == "cells":
            return buf.view(np.int32).reshape(-1, 8)
        if what == "gcells":
            return buf.view(np.float64).reshape(-1, 8)
        if what == "ccells":
            v = buf.view(np.float64)
            nc = len(v) // 5
            return v[: 4 * nc].reshape(-1, 4), v[4 * nc:]
        if what in ("multipoles", "local"):
            return buf.view(np.float64)
        return buf.view(np.int32).reshape(-1, 2)

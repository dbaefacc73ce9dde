"""The allocation-free step (ncorp_step_noalloc: the workspace is a fixed array
inside the library, one per GPU) against ncorp_step on a caller workspace: same
kernels, so the states and the collision pairs must agree bit for bit.  Several
calls in a row share the one array; each must start from cleared state, so a
second, smaller input, another context and the mesh module (whose device state
persists between builds on a workspace) follow each other here."""
import numpy as np
import pytest

from paper_2310_20374_amd import inputs
from tests.gpu_util import dev_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nc():
    from paper_2310_20374_amd import ncorp
    ncorp.lib()
    return ncorp


def _run(nc, d, prm, dt, n_steps, noalloc, ctx=None, cap=1 << 15):
    import torch
    n = len(d["x"])
    if ctx is None:
        ctx = nc.Context(prm, 0 if noalloc else n, pair_capacity=cap)
    t = dev_arrays(d)
    pairs = torch.zeros((cap, 3), dtype=torch.int64, device="cuda:0")
    npairs = torch.zeros(n_steps, dtype=torch.int64, device="cuda:0")
    args = (t["x"], t["y"], t["z"], t["vx"], t["vy"], t["vz"], t["m"], t["R"], dt, n_steps,
            pairs, npairs)
    if noalloc:
        ctx.step_noalloc(*args)
    else:
        ctx.step(*args)
    torch.cuda.synchronize()
    ctx.check_status()
    cnt = npairs.cpu().numpy()
    out = {k: t[k].cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    return ctx, out, pairs[: int(cnt.sum())].cpu().numpy(), cnt


def _same(a, b):
    _, sa, pa, ca = a
    _, sb, pb, cb = b
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
    assert np.array_equal(ca, cb)
    assert np.array_equal(pa, pb)


def test_noalloc_matches_step_on_two_calls_in_a_row(nc):
    # call 1: clustered input with collisions, p = 4
    d1 = inputs.clumps(6000, seed=5, n_clumps=10)
    prm1 = nc.params_default(4, leaf_size=16)
    print("noalloc call 1: clumps n=6000 p=4 s=16, 3 steps", flush=True)
    ref1 = _run(nc, d1, prm1, 2e-3, 3, noalloc=False)
    got1 = _run(nc, d1, prm1, 2e-3, 3, noalloc=True)
    _same(got1, ref1)
    assert ref1[3].sum() > 0
    # call 2: a smaller input on another context and order, p = 3
    d2 = inputs.disk(2500, seed=6)
    prm2 = nc.params_default(3, leaf_size=16)
    print("noalloc call 2: disk n=2500 p=3 s=16, 2 steps", flush=True)
    ref2 = _run(nc, d2, prm2, 1e-3, 2, noalloc=False)
    got2 = _run(nc, d2, prm2, 1e-3, 2, noalloc=True)
    _same(got2, ref2)
    # call 3: the first context again, now on a smaller input than its own last call
    d3 = inputs.clumps(4000, seed=7, n_clumps=6)
    print("noalloc call 3: clumps n=4000 on the first context", flush=True)
    ref3 = _run(nc, d3, prm1, 2e-3, 2, noalloc=False)
    got3 = _run(nc, d3, prm1, 2e-3, 2, noalloc=True, ctx=got1[0])
    _same(got3, ref3)


def test_noalloc_mesh_module_after_tree_calls(nc):
    """The mesh keeps device state between builds on one workspace; on the shared
    array it must restart from Eq. (4) like on a new workspace, call after call."""
    prm = nc.params_default(3, gravity_method=nc.GRAVITY_MESH,
                            collision_method=nc.COLLISIONS_MESH, mesh_cells=64,
                            mesh_neighbours=6.0, mesh_aspect=0.05)
    for k, n in enumerate((3000, 1800)):
        d = inputs.gas_box(n, seed=11 + k, radius=0.01)
        print(f"noalloc mesh call {k}: gas box n={n}", flush=True)
        ref = _run(nc, d, prm, 2e-3, 3, noalloc=False)
        got = _run(nc, d, prm, 2e-3, 3, noalloc=True)
        _same(got, ref)

"""GPU parity of the tree build and the climbs against the CPU oracle:
Hilbert keys, permutation and flat-tree topology bit for bit (Sect. 3.4.1,
3.4.6); centres, masses, r_max, r_crit and opening angles of the gravity climb
(Eqs. 10-12) and the collision climb (Eqs. 7-9) bit for bit; multipole moments
(Eq. 20 / App. C) to rounding."""
import math

import numpy as np
import pytest

from paper_2310_20374_amd import inputs
from tests.gpu_util import dev_arrays

pytestmark = pytest.mark.gpu

CASES = {
    "disk2k_s16": (lambda: inputs.disk(2000, seed=0), 16),
    "disk1e5_s52": (lambda: inputs.disk(100000, seed=0), 52),
    "clumps2e4_s16": (lambda: inputs.clumps(20000, seed=0, n_clumps=20), 16),
    "gas3k_s8": (lambda: inputs.gas_box(3000, seed=0), 8),
    "disk3k_s1": (lambda: inputs.disk(3000, seed=1), 1),
    "tiny_root_leaf": (lambda: inputs.disk(40, seed=2), 64),
    "single": (lambda: inputs.disk(1, seed=3), 16),
    "ragged_4097": (lambda: inputs.hot_disk(4097, seed=4), 17),
    # every position three times, 43 moonlets on one point: a leaf at the depth cap
    "coincident3k_s16": (lambda: inputs.coincident(3000, seed=5), 16),
}


@pytest.fixture(scope="module")
def nc():
    from paper_2310_20374_amd import ncorp
    ncorp.lib()
    return ncorp


def _build(nc, d, s, p=3):
    import torch
    prm = nc.params_default(p, leaf_size=s)
    ctx = nc.Context(prm, len(d["x"]), pair_capacity=1 << 18)
    t = dev_arrays(d)
    ctx.build_tree(t["x"], t["y"], t["z"])
    torch.cuda.synchronize()
    ctx.check_status()
    return ctx, t


@pytest.mark.parametrize("case", list(CASES))
def test_keys_perm_topology(nc, orc, case):
    gen, s = CASES[case]
    d = gen()
    print(f"case {case} n={len(d['x'])} s={s}", flush=True)
    ctx, _ = _build(nc, d, s)
    t = orc.Tree(d["x"], d["y"], d["z"], s)
    info = ctx.tree_info()
    assert info["ncells"] == t.ncells
    assert info["nleaves"] == int((t.nchild == 0).sum())
    assert info["maxlevel"] == t.maxlevel
    keys = ctx.export("keys")
    perm = ctx.export("perm").astype(np.int64)
    assert np.array_equal(perm, t.perm)
    assert np.array_equal(keys, t.keys[t.perm])
    cells = ctx.export("cells")
    assert np.array_equal(cells[:, 0], t.level)
    assert np.array_equal(cells[:, 1], t.first)
    assert np.array_equal(cells[:, 2], t.count)
    assert np.array_equal(cells[:, 3], t.child_first)
    assert np.array_equal(cells[:, 4], t.nchild)
    assert np.array_equal(cells[:, 5], t.parent)
    pref = cells[:, 6].astype(np.uint32).astype(np.uint64) | (
        cells[:, 7].astype(np.uint32).astype(np.uint64) << np.uint64(32))
    assert np.array_equal(pref, t.prefix)


def _sym_from_full(full, n):
    """Scaled symmetric components M_a / a! of a full order-n tensor, in the
    library's order (ax descending, then ay descending)."""
    out = []
    T = full.reshape((3,) * n) if n else full.reshape(())
    for bc in range(n + 1):          # a = n - bc descending
        for c in range(bc + 1):       # then b = bc - c descending
            b = bc - c
            a = n - bc
            idx = (0,) * a + (1,) * b + (2,) * c
            v = T[idx] if n else float(T)
            out.append(v / (math.factorial(a) * math.factorial(b) * math.factorial(c)))
    return np.array(out)


@pytest.mark.parametrize("case", ["disk2k_s16", "clumps2e4_s16", "disk1e5_s52"])
@pytest.mark.parametrize("p", [3, 6])
def test_gravity_climb(nc, orc, case, p):
    import torch
    gen, s = CASES[case]
    d = gen()
    print(f"case {case} p={p}", flush=True)
    ctx, t = _build(nc, d, s, p)
    n = len(d["x"])
    a = [torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    ctx.gravity(t["m"], *a)
    torch.cuda.synchronize()
    ctx.check_status()
    tr = orc.Tree(d["x"], d["y"], d["z"], s)
    g = orc.Gravity(tr, d["m"], 1.0, p, 0.5, 0)
    ref = g.cells()
    gc = ctx.export("gcells")
    # bit-exact: same operations in the same order on both sides
    assert np.array_equal(gc[:, 0:3], ref["s"])
    assert np.array_equal(gc[:, 3], ref["mass"])
    assert np.array_equal(gc[:, 4], ref["rmax"])
    assert np.array_equal(gc[:, 5], ref["rcrit"])
    # multipole moments: App. C shifts on the GPU vs Eq. (20) sums in the oracle
    nm = ctx.export("multipoles").reshape(tr.ncells, -1)
    orders = [0] + list(range(2, p))
    for c in range(0, tr.ncells, max(1, tr.ncells // 200)):
        Mfull, _ = g.cell_tensors(c)
        off, col = 0, 0
        for k in orders:
            blk = Mfull[off: off + 3 ** k]
            off += 3 ** k
            want = _sym_from_full(blk, k)
            got = nm[c, col: col + len(want)]
            col += len(want)
            scale = np.abs(want).max() + 1e-300
            assert np.abs(got - want).max() <= 1e-11 * scale, (c, k)


@pytest.mark.parametrize("case", ["gas3k_s8", "clumps2e4_s16", "disk2k_s16"])
def test_collision_climb(nc, orc, case):
    import torch
    gen, s = CASES[case]
    d = gen()
    dt = 0.05
    ctx, t = _build(nc, d, s)
    pairs = torch.zeros((1 << 18, 2), dtype=torch.int64, device="cuda:0")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    ctx.collide(t["vx"], t["vy"], t["vz"], t["R"], dt, pairs, npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    tr = orc.Tree(d["x"], d["y"], d["z"], s)
    co = orc.Collide(tr, d["vx"], d["vy"], d["vz"], d["R"], dt)
    ref = co.cells()
    cc, rmax = ctx.export("ccells")
    assert np.array_equal(cc[:, 0:3], ref["sbar"])
    assert np.array_equal(cc[:, 3], ref["rcrit"])
    assert np.array_equal(rmax, ref["rmax"])

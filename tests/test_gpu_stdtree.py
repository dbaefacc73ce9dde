"""GPU parity of the standard tree code (Alg. 1, Sect. 3.4.4): accelerations equal
to the oracle's standard tree to FP64 rounding on the same tree and thresholds,
the direct-sum limit, the p = 1 / p = 2 identity, ragged sizes, and forests of
disks equal to the per-disk calls bit for bit."""
import numpy as np
import pytest

from paper_2310_20374_amd import inputs
from tests.gpu_util import dev_arrays, rel_err, run_gravity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nc():
    from paper_2310_20374_amd import ncorp
    ncorp.lib()
    return ncorp


def _prm(nc, p, s=102, pre=6, post=16, mode=0, theta=0.5):
    return nc.params_default(p, leaf_size=s, gravity_method=nc.GRAVITY_STANDARD_TREE,
                             ncb_pre=pre, ncb_post=post, theta_mode=mode, theta_min=theta)


STD_CASES = {
    # name: (generator, p, s, (ncb_pre, ncb_post), theta_mode, theta_min)
    "disk2e4_p3_paper": (lambda: inputs.disk(20000, seed=3), 3, 102, (6, 16), 0, 0.5),
    "disk8k_p6": (lambda: inputs.disk(8000, seed=4), 6, 102, (6, 16), 0, 0.5),
    "disk3k_p1": (lambda: inputs.disk(3000, seed=5), 1, 16, (6, 16), 0, 0.5),
    "clumps2e4_p4_const_theta": (lambda: inputs.clumps(20000, seed=1, n_clumps=20), 4, 32,
                                 (6, 16), 1, 0.6),
    "hot6k_p5_no_thresholds": (lambda: inputs.hot_disk(6000, seed=2), 5, 8, (0, 0), 0, 0.5),
    "disk5e3_p2_wide_thresholds": (lambda: inputs.disk(5000, seed=6), 2, 64, (64, 200), 0, 0.3),
    "gas1e4_p3_s1": (lambda: inputs.gas_box(10000, seed=7), 3, 1, (1, 1), 0, 0.5),
    # equal positions: zero-distance pairs and a leaf at the depth cap
    "coincident3k_p4": (lambda: inputs.coincident(3000, seed=5), 4, 16, (6, 16), 0, 0.5),
}


@pytest.mark.parametrize("case", list(STD_CASES))
def test_standard_tree_matches_oracle(nc, orc, case):
    gen, p, s, (pre, post), mode, theta = STD_CASES[case]
    d = gen()
    print(f"case {case}", flush=True)
    _, a = run_gravity(nc, d, _prm(nc, p, s, pre, post, mode, theta))
    ref, _, _ = orc.standard_tree_accel(d, p=p, s=s, ncb_pre=pre, ncb_post=post,
                                        theta_mode=mode, theta_min=theta)
    rms, mx = rel_err(a, ref)
    assert mx < 1e-11, (rms, mx)


@pytest.mark.parametrize("n", [1, 2, 63, 65, 1000, 4097])
def test_ragged_sizes(nc, orc, n):
    """Sizes that leave a wave partly empty, a single moonlet (zero acceleration)
    and a root that is a leaf."""
    d = inputs.disk(n, seed=11)
    print(f"n {n}", flush=True)
    _, a = run_gravity(nc, d, _prm(nc, 3, s=16))
    if n == 1:
        assert np.all(a == 0.0)
        return
    ref, _, _ = orc.standard_tree_accel(d, p=3, s=16)
    assert rel_err(a, ref)[1] < 1e-11


def test_pre_threshold_above_n_is_direct_sum(nc, orc):
    d = inputs.disk(3000, seed=12)
    _, a = run_gravity(nc, d, _prm(nc, 3, pre=10 ** 9))
    ref = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    assert rel_err(a, ref)[1] < 1e-12


def test_p1_equals_p2(nc):
    """The dipole vanishes about the centre of mass (Sect. 3.4.2): p = 1 and p = 2
    are the same standard tree code."""
    d = inputs.disk(8000, seed=13)
    _, a1 = run_gravity(nc, d, _prm(nc, 1))
    _, a2 = run_gravity(nc, d, _prm(nc, 2))
    assert np.array_equal(a1, a2)


def test_precision_flag_does_not_apply(nc):
    """The standard tree computes in FP64 whatever the precision flag says."""
    d = inputs.disk(5000, seed=14)
    _, a = run_gravity(nc, d, _prm(nc, 4))
    prm = _prm(nc, 4)
    prm.precision = nc.FP32_BULK
    _, b = run_gravity(nc, d, prm)
    assert np.array_equal(a, b)


def test_forest_equals_per_disk(nc, orc):
    """A batched tree of disks: each disk's moonlets walk their own tree only; the
    result is bit-identical to the plain call on that disk alone."""
    import torch
    sizes = [2000, 1, 0, 40, 3001, 17, 5000, 0]
    d, off = inputs.disk_batch(sizes)
    n = len(d["x"])
    prm = _prm(nc, 3, s=16)
    ctx = nc.Context(prm, n, pair_capacity=1 << 14, device="cuda:0")
    t = dev_arrays(d)
    offd = torch.tensor(off, device="cuda:0")
    a = [torch.empty(n, dtype=torch.float64, device="cuda:0") for _ in range(3)]
    ctx.build_tree_batched(offd, t["x"], t["y"], t["z"])
    ctx.gravity(t["m"], *a)
    torch.cuda.synchronize()
    ctx.check_status()
    a = torch.stack(a, 1).cpu().numpy()
    for k in range(len(sizes)):
        part = {key: v[off[k]:off[k + 1]] for key, v in d.items()}
        nk = len(part["x"])
        if nk == 0:
            continue
        got = a[off[k]:off[k + 1]]
        _, plain = run_gravity(nc, part, prm)
        assert np.array_equal(got, plain), k
        if nk > 1:
            ref, _, _ = orc.standard_tree_accel(part, p=3, s=16)
            assert rel_err(got, ref)[1] < 1e-11, k


def test_step_with_standard_tree(nc, orc):
    """ncorp_step driven by the standard tree: one KDK step equals the oracle's
    leapfrog with the oracle standard tree as its acceleration."""
    import torch
    d = inputs.disk(4000, seed=15)
    n = len(d["x"])
    dt = 1e-3
    prm = _prm(nc, 3, s=32)
    ctx = nc.Context(prm, n, pair_capacity=1 << 14, device="cuda:0")
    t = dev_arrays(d)
    pairs = torch.zeros((1 << 14, 3), dtype=torch.int64, device="cuda:0")
    npairs = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    ctx.step(t["x"], t["y"], t["z"], t["vx"], t["vy"], t["vz"], t["m"], t["R"], dt, 2, pairs,
             npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    ref, _ = orc.kdk_steps(d, dt, 2, lambda s: orc.standard_tree_accel(s, p=3, s=32)[0])
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        got = t[k].cpu().numpy()
        assert np.abs(got - ref[k]).max() < 1e-11, k


# ---------------------------------------------------------------- collisions
from tests.gpu_util import run_collide  # noqa: E402

COL_CASES = {
    # name: (generator, dt, leaf size, (ncb_pre, ncb_post))
    "gas2k_s8": (lambda: inputs.gas_box(2000, seed=1), 0.01, 8, (6, 16)),
    "gas2k_s102_no_thresholds": (lambda: inputs.gas_box(2000, seed=3), 0.01, 102, (0, 0)),
    "disk3k_dt2": (lambda: inputs.disk(3000, seed=2), 2.0, 16, (6, 16)),
    "hot3k_wide": (lambda: inputs.hot_disk(3000, seed=0), 0.5, 17, (64, 200)),
    "clumps2e4_s102": (lambda: inputs.clumps(20000, seed=0, n_clumps=20), 0.01, 102, (6, 16)),
    "clumps2e4_s1": (lambda: inputs.clumps(20000, seed=1, n_clumps=20), 0.01, 1, (1, 1)),
}


@pytest.mark.parametrize("case", list(COL_CASES))
def test_standard_tree_collisions_equal_brute_force(nc, orc, case):
    """Alg. 1 in its collision form finds exactly the brute-force pairs (Sect. 3.1)."""
    gen, dt, s, (pre, post) = COL_CASES[case]
    d = gen()
    print(f"case {case}", flush=True)
    prm = nc.params_default(3, leaf_size=s, collision_method=nc.COLLISIONS_STANDARD_TREE,
                            ncb_pre=pre, ncb_post=post)
    _, pairs = run_collide(nc, d, prm, dt)
    want = orc.pairs_brute(d, dt)
    assert len(want) > 0
    assert np.array_equal(pairs, want)


def test_standard_tree_collisions_forest(nc, orc):
    import torch
    sizes = [2000, 1, 0, 40, 3001, 17]
    d, off = inputs.disk_batch(sizes)
    n = len(d["x"])
    prm = nc.params_default(3, leaf_size=16, collision_method=nc.COLLISIONS_STANDARD_TREE)
    ctx = nc.Context(prm, n, pair_capacity=1 << 16, device="cuda:0")
    t = dev_arrays(d)
    offd = torch.tensor(off, device="cuda:0")
    pairs = torch.zeros((1 << 16, 2), dtype=torch.int64, device="cuda:0")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    ctx.build_tree_batched(offd, t["x"], t["y"], t["z"])
    ctx.collide(t["vx"], t["vy"], t["vz"], t["R"], 5.0, pairs, npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    got = pairs[: int(npairs.item())].cpu().numpy()
    want = []
    for k in range(len(sizes)):
        part = {key: v[off[k]:off[k + 1]] for key, v in d.items()}
        if len(part["x"]) > 1:
            want.append(orc.pairs_brute(part, 5.0) + off[k])
    want = np.concatenate(want)
    want = want[np.lexsort((want[:, 1], want[:, 0]))]
    assert len(want) > 20
    assert np.array_equal(got, want)


def test_step_standard_tree_everywhere(nc, orc):
    """ncorp_step with the standard tree for gravity and collisions, elastic resolution:
    states and resolved pairs against the oracle's leapfrog with its standard tree and
    brute-force pairs."""
    import torch
    d = inputs.clumps(4000, seed=2, n_clumps=8)
    n, dt, ns = len(d["x"]), 2e-3, 3
    prm = nc.params_default(3, leaf_size=32, gravity_method=nc.GRAVITY_STANDARD_TREE,
                            collision_method=nc.COLLISIONS_STANDARD_TREE,
                            collision_mode=nc.COLLISIONS_RESOLVE)
    ctx = nc.Context(prm, n, pair_capacity=1 << 16, device="cuda:0")
    t = dev_arrays(d)
    pairs = torch.zeros((1 << 16, 3), dtype=torch.int64, device="cuda:0")
    npairs = torch.zeros(ns, dtype=torch.int64, device="cuda:0")
    ctx.step(t["x"], t["y"], t["z"], t["vx"], t["vy"], t["vz"], t["m"], t["R"], dt, ns, pairs,
             npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    ref, ref_pairs = orc.kdk_steps(d, dt, ns, lambda s: orc.standard_tree_accel(s, p=3, s=32)[0],
                                   collide_fn=orc.pairs_brute, resolve_f=2.0)
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        assert np.abs(t[k].cpu().numpy() - ref[k]).max() < 1e-11, k
    cnt = npairs.cpu().numpy()
    got = pairs[: int(cnt.sum())].cpu().numpy()
    off = 0
    for step in range(ns):
        mine = got[off: off + cnt[step]]
        off += cnt[step]
        assert np.array_equal(mine[:, 1:], ref_pairs[step]), step
    assert cnt.sum() > 0

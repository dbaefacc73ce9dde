"""GPU leapfrog (Sect. 4.1, merged kick-drift-kick around the central mass of
App. B.1) against the oracle integrator driven by the oracle tree: positions and
velocities to FP64 rounding after several steps, and each step's collision pairs
(searched on (x_n, v_n+1/2) over dt) bit for bit."""
import math

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


def _gpu_steps(nc, d, prm, dt, n_steps, cap=1 << 16):
    import torch
    n = len(d["x"])
    ctx = nc.Context(prm, n, pair_capacity=cap)
    t = dev_arrays(d)
    pairs = torch.zeros((cap, 3), dtype=torch.int64, device="cuda:0")
    npairs = torch.zeros(n_steps, dtype=torch.int64, device="cuda:0")
    ctx.step(t["x"], t["y"], t["z"], t["vx"], t["vy"], t["vz"], t["m"], t["R"], dt, n_steps,
             pairs, npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    out = {k: t[k].cpu().numpy() for k in ("x", "y", "z", "vx", "vy", "vz")}
    cnt = npairs.cpu().numpy()
    return out, pairs[: int(cnt.sum())].cpu().numpy(), cnt


def _oracle_steps(orc, d, prm, dt, n_steps):
    def accel(s):
        a, _, _ = orc.tree_accel(s, G=prm.G, p=prm.p, theta_min=prm.theta_min, s=prm.leaf_size,
                                 ncs=prm.ncs, ncc_pre=prm.ncc_pre, ncc_post=prm.ncc_post,
                                 theta_mode=prm.theta_mode)
        return a

    def collide(s, h):
        return orc.pairs_brute(s, h)

    return orc.kdk_steps(d, dt, n_steps, accel if prm.p > 0 else None, G=prm.G,
                         M_central=prm.M_central, collide_fn=collide)


@pytest.mark.parametrize("case", ["disk2k_p3", "clumps4k_p4"])
def test_steps_match_oracle(nc, orc, case):
    if case == "disk2k_p3":
        d, prm, dt, ns = inputs.disk(2000, seed=0), nc.params_default(3, leaf_size=16), 1e-3, 5
    else:
        d = inputs.clumps(4000, seed=2, n_clumps=8)
        prm, dt, ns = nc.params_default(4, leaf_size=16), 2e-3, 3
    print(f"case {case}", flush=True)
    got, pairs, cnt = _gpu_steps(nc, d, prm, dt, ns)
    ref, ref_pairs = _oracle_steps(orc, d, prm, dt, ns)
    for k in ("x", "y", "z"):
        assert np.abs(got[k] - ref[k]).max() < 1e-12 * 10.0, k
    for k in ("vx", "vy", "vz"):
        assert np.abs(got[k] - ref[k]).max() < 1e-11, k
    off = 0
    for step in range(ns):
        mine = pairs[off: off + cnt[step]]
        off += cnt[step]
        assert np.all(mine[:, 0] == step)
        assert np.array_equal(mine[:, 1:], ref_pairs[step]), step
    if case == "clumps4k_p4":
        assert cnt.sum() > 0


def test_kepler_orbit(nc, orc):
    """One moonlet, no mutual gravity: a Kepler orbit to O(dt^2)."""
    d = {"x": np.array([3.0]), "y": np.array([0.0]), "z": np.array([0.0]),
         "vx": np.array([0.0]), "vy": np.array([math.sqrt(1 / 3.0) * 1.1]),
         "vz": np.array([0.0]), "m": np.array([1e-9]), "R": np.array([0.01])}
    prm = nc.params_default(0)
    period = 2 * math.pi * (1.0 / (2 / 3.0 - (1 / 3.0) * 1.21)) ** 1.5
    dt = period / 400
    got, _, cnt = _gpu_steps(nc, d, prm, dt, 400, cap=16)
    ref, _ = orc.kdk_steps(d, dt, 400, None)
    for k in got:
        assert abs(got[k][0] - ref[k][0]) < 1e-11, k
    assert abs(got["x"][0] - 3.0) < 50 * dt * dt
    assert np.all(cnt == 0)

"""GPU kicks with the central-body extras (App. B: J2 bulge, quadrupolar tide of a
distant body on a tilted circular orbit) against the oracle's leapfrog, with and
without mutual gravity, and the context clock across calls."""
import numpy as np
import pytest

from paper_2310_20374_amd import inputs
from tests.gpu_util import dev_arrays

pytestmark = pytest.mark.gpu

FIELDS = ("x", "y", "z", "vx", "vy", "vz")
EXTRA = dict(J2=1.08e-3, R_central=1.0, M_sun=332946.0, a_sun=23481.0, obliquity=0.4091)


@pytest.fixture(scope="module")
def nc():
    from paper_2310_20374_amd import ncorp
    ncorp.lib()
    return ncorp


def _gpu(nc, d, prm, dt, calls):
    import torch
    ctx = nc.Context(prm, len(d["x"]), pair_capacity=1 << 12)
    t = dev_arrays(d)
    for ns in calls:
        pairs = torch.zeros((1 << 12, 3), dtype=torch.int64, device="cuda:0")
        npairs = torch.zeros(ns, dtype=torch.int64, device="cuda:0")
        ctx.step(t["x"], t["y"], t["z"], t["vx"], t["vy"], t["vz"], t["m"], t["R"], dt, ns,
                 pairs, npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    return {k: t[k].cpu().numpy() for k in FIELDS}


@pytest.mark.parametrize("p", [0, 3])
def test_steps_with_central_extras_match_oracle(nc, orc, p):
    d = inputs.disk(2000, seed=4)
    dt, ns, t0 = 5e-3, 6, 123.0
    prm = nc.params_default(p, leaf_size=16, t_start=t0, **EXTRA)
    got = _gpu(nc, d, prm, dt, [ns])

    accel = None
    if p > 0:
        def accel(s):
            return orc.tree_accel(s, p=p, s=16, ncs=prm.ncs, ncc_pre=prm.ncc_pre,
                                  ncc_post=prm.ncc_post)[0]
    ref, _ = orc.kdk_steps(d, dt, ns, accel, central=EXTRA, t_start=t0)
    # the extras change the orbit measurably over the run
    plain, _ = orc.kdk_steps(d, dt, ns, accel, t_start=t0)
    assert np.abs(ref["vz"] - plain["vz"]).max() > 1e-8
    for k in ("x", "y", "z"):
        assert np.abs(got[k] - ref[k]).max() < 1e-12 * 10.0, k
    for k in ("vx", "vy", "vz"):
        assert np.abs(got[k] - ref[k]).max() < 1e-11, k


def test_clock_continues_across_calls(nc):
    """Two calls of three steps follow one call of six (the distant body's longitude
    keeps advancing with the context clock)."""
    d = inputs.disk(1500, seed=6)
    prm = nc.params_default(0, t_start=50.0, **EXTRA)
    one = _gpu(nc, d, prm, 0.01, [6])
    two = _gpu(nc, d, prm, 0.01, [3, 3])
    for k in FIELDS:
        assert np.abs(one[k] - two[k]).max() < 1e-13, k

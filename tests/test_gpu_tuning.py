"""Launch-shape parameters of the gravity evaluation and the autotuner that picks them.

The direct sums' tile shape (p2p_tile, p2p_targets_max) only regroups the same
per-target sums, and the number of walk waves only changes the order in which the
walk's lists fill (every consumer sorts them), so the accelerations stay those of the
oracle tree and, for the walk, bit-identical.  The tuner keeps the fastest candidate
whose error passes its gate."""
import numpy as np
import pytest

from paper_2310_20374_amd import inputs
from tests.gpu_util import dev_arrays, run_gravity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nc():
    from paper_2310_20374_amd import ncorp
    ncorp.lib()
    return ncorp


def _rel(a, b):
    return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_launch_shape_keeps_the_accelerations(nc, orc, precision):
    d = inputs.disk(20000, seed=7)
    prec = nc.FP64 if precision == "fp64" else nc.FP32_BULK
    prm0 = nc.params_default(4, leaf_size=48, precision=prec)
    base = dict(leaf_size=48, precision=prec)
    _, a0 = run_gravity(nc, d, prm0)
    ref, _, _ = orc.tree_accel(d, p=4, s=48, ncs=prm0.ncs, ncc_pre=prm0.ncc_pre,
                               ncc_post=prm0.ncc_post)
    tol = 1e-11 if precision == "fp64" else 1e-4
    assert _rel(a0, ref) < tol
    for tile, tmax in ((128, 4), (512, 4), (256, 1), (256, 2), (512, 3)):
        print(f"{precision} tile {tile} targets {tmax}", flush=True)
        _, a = run_gravity(nc, d, nc.params_default(4, p2p_tile=tile, p2p_targets_max=tmax,
                                                    **base))
        assert _rel(a, ref) < tol
        if precision == "fp64":
            assert _rel(a, a0) < 1e-13
    for waves in (256, 512, 2048):
        print(f"{precision} walk waves {waves}", flush=True)
        _, a = run_gravity(nc, d, nc.params_default(4, walk_waves=waves, **base))
        assert np.array_equal(a, a0)


def test_tuner_keeps_the_fastest_candidate_that_passes(nc):
    import torch
    from paper_2310_20374_amd import autotune
    d = inputs.disk(30000, seed=8)
    base = dev_arrays(d)
    prm = nc.params_default(4, precision=nc.FP32_BULK)
    tuned, tab = autotune.tune_step(nc, prm, base, steps=2, leaf_sizes=(32, 64),
                                    tile_shapes=((256, 4), (128, 2)), walk_waves=(1024, 512),
                                    samples=1024)
    for stage, key in (("leaf_size", tuned.leaf_size),
                       ("p2p_tile_x_targets_max", f"{tuned.p2p_tile}x{tuned.p2p_targets_max}"),
                       ("walk_waves", tuned.walk_waves)):
        rows = tab[stage]
        assert rows[key]["passed"]
        fastest = min((k for k in rows if rows[k]["passed"]), key=lambda k: rows[k]["ms_per_step"])
        assert fastest == key
        assert all(r["gate_error"] < 1e-4 for r in rows.values())
    # a gate nothing can pass: the most accurate candidate is kept, marked as failing
    tuned, tab = autotune.tune_step(nc, prm, base, steps=1, leaf_sizes=(32, 64),
                                    tile_shapes=((256, 4),), walk_waves=(1024,), gate=1e-14,
                                    samples=512)
    rows = tab["leaf_size"]
    assert not any(r["passed"] for r in rows.values())
    assert tuned.leaf_size == min(rows, key=lambda k: rows[k]["gate_error"])
    torch.cuda.synchronize()

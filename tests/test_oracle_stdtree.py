"""Pins of the oracle's standard tree code (Alg. 1, Sect. 3.4.4; cell-moonlet terms
of Sect. 3.4.2): limits that reduce it to the direct sum, the p = 1 / p = 2
identity the paper states, and the truncation error of the C^(1) series on a
moonlet far from a compact group, order by order."""
import numpy as np
import pytest

from paper_2310_20374_amd import inputs


def _rel(a, b):
    return np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)


def test_pre_threshold_above_n_is_direct_sum(orc):
    """N_cb,pre above N: the root itself is summed moonlet by moonlet."""
    d = inputs.disk(1500, seed=21)
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    a, _, _ = orc.standard_tree_accel(d, p=3, ncb_pre=10**9)
    assert np.abs(a - ex).max() <= 1e-13 * np.abs(ex).max()


def test_huge_opening_radius_is_direct_sum(orc):
    """theta -> 0 (r_crit -> infinity): no cell is ever well separated, every
    moonlet ends up summed directly at the leaves or below N_cb,post."""
    d = inputs.disk(1500, seed=22)
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    a, _, _ = orc.standard_tree_accel(d, p=3, theta_min=1e-9, theta_mode=1, s=8)
    assert np.abs(a - ex).max() <= 1e-13 * np.abs(ex).max()


def test_p1_equals_p2(orc):
    """The dipole vanishes about the centre of mass, so p = 1 and p = 2 give the
    same accelerations in the standard tree code (Sect. 3.4.2)."""
    d = inputs.disk(3000, seed=23)
    a1, _, _ = orc.standard_tree_accel(d, p=1)
    a2, _, _ = orc.standard_tree_accel(d, p=2)
    assert np.array_equal(a1, a2)
    a3, _, _ = orc.standard_tree_accel(d, p=3)
    assert not np.array_equal(a1, a3)


def _far_group(n=400, r=0.05, D=4.0, seed=5):
    """A compact random group of radius r at the origin and one moonlet at
    distance D; the group's moonlets have unequal masses so that every multipole
    order is present."""
    rng = np.random.default_rng(seed)
    u = rng.normal(size=(n, 3))
    u *= (r * rng.random(n) ** (1 / 3) / np.linalg.norm(u, axis=1))[:, None]
    u[:, 0] *= 1.6                                   # anisotropic: odd and even orders
    u[:, 2] *= 0.5
    pos = np.vstack([u, [[D * 0.6, D * 0.64, D * 0.48]]])
    m = np.concatenate([rng.random(n) * 1e-6 + 1e-7, [1e-7]])
    z = np.zeros(n + 1)
    return {"x": pos[:, 0], "y": pos[:, 1], "z": pos[:, 2], "vx": z, "vy": z, "vz": z,
            "m": m, "R": z + 1e-4}, r / D


def test_far_moonlet_truncation_error_by_order(orc):
    """The far moonlet sees the group through C^(1) terms only; the error of the
    series cut after order n = p - 1 falls like (r/D)^max(p, 2), so a dropped or
    mis-signed term of any order up to 5 shows up as an error one order larger."""
    d, eps = _far_group()
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])[-1]
    errs = {}
    for p in range(1, 7):
        a, _, _ = orc.standard_tree_accel(d, p=p, s=32, ncb_pre=6, ncb_post=16)
        errs[p] = np.linalg.norm(a[-1] - ex) / np.linalg.norm(ex)
        assert errs[p] <= 3.0 * eps ** max(p, 2), (p, errs[p])
    # p = 3 and up actually improve on the previous order
    for p in range(3, 7):
        assert errs[p] < 0.2 * errs[p - 1], errs


def test_errors_fall_with_order_on_a_disk(orc):
    """Median relative error against the direct sum on a disk (Fig. 5 behaviour):
    higher orders are more precise, and p = 6 is well below one percent."""
    d = inputs.disk(4000, seed=24)
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    med = {}
    for p in (1, 3, 6):
        a, _, _ = orc.standard_tree_accel(d, p=p)
        med[p] = float(np.median(_rel(a, ex)))
    assert med[6] < med[3] < med[1]
    assert med[6] < 2e-3


@pytest.mark.parametrize("pre,post", [(6, 16), (1, 1), (64, 200)])
def test_thresholds_do_not_change_far_field_exactness(orc, pre, post):
    """Whatever the thresholds, the sum of all contributions is the direct sum up to
    the expansion error: with p = 6 and a small opening angle the thresholds only
    move work between the two exact-enough forms."""
    d = inputs.disk(2000, seed=25)
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    a, _, _ = orc.standard_tree_accel(d, p=6, theta_min=0.2, theta_mode=1, ncb_pre=pre,
                                      ncb_post=post)
    assert np.median(_rel(a, ex)) < 1e-6


def test_zero_thresholds_stay_finite(orc):
    """N_cb,pre = N_cb,post = 0 on small leaves: single-moonlet cells have r_crit = 0
    and are not separated from their own moonlet (reading of the MAC at x = s_B);
    the result is finite and as precise as with the paper's thresholds."""
    d = inputs.hot_disk(3000, seed=2)
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    a, _, _ = orc.standard_tree_accel(d, p=5, s=8, ncb_pre=0, ncb_post=0)
    assert np.all(np.isfinite(a))
    b, _, _ = orc.standard_tree_accel(d, p=5, s=8)
    assert np.median(_rel(a, ex)) < 3 * np.median(_rel(b, ex))


def test_sampled_walks_equal_full_run(orc):
    """The per-target entry point gives the full run's values for those moonlets."""
    d = inputs.disk(3000, seed=26)
    a, _, g = orc.standard_tree_accel(d, p=4, s=32)
    tg = np.array([0, 17, 999, 2999, 1500])
    assert np.array_equal(g.standard_targets(6, 16, tg), a[tg])

"""Pins of the oracle's collision resolution (Sect. 5.1 hard-sphere impulse, Sect. 5.2
inelastic coefficient f; one collision per moonlet and step, the earliest first):
closed forms and invariants that do not re-type the oracle's own arithmetic."""
import math

import numpy as np
import pytest

from paper_2310_20374_amd import inputs


def _state(rows):
    keys = ("x", "y", "z", "vx", "vy", "vz", "m", "R")
    return {k: np.array([r[i] for r in rows], dtype=np.float64) for i, k in enumerate(keys)}


def _drift(s, dt):
    for a, v in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        s[a] = s[a] + dt * s[v]


def test_head_on_equal_masses_elastic_exchange(orc):
    """Equal masses, head on, f = 2: the velocities are exchanged at contact, and the
    moonlets end where the piecewise-straight motion puts them."""
    s = _state([(-0.05, 0, 0, 1.0, 0, 0, 1e-6, 0.01), (0.05, 0, 0, -1.0, 0, 0, 1e-6, 0.01)])
    res = orc.resolve(s, [[0, 1]], 0.1, 2.0)
    assert res.tolist() == [[0, 1]]
    assert s["vx"][0] == pytest.approx(-1.0, abs=1e-14)
    assert s["vx"][1] == pytest.approx(1.0, abs=1e-14)
    _drift(s, 0.1)
    # contact at t = (0.1 - 0.02) / 2 = 0.04 at x = -0.01 and +0.01, then 0.06 back out
    assert s["x"][0] == pytest.approx(-0.07, abs=1e-14)
    assert s["x"][1] == pytest.approx(0.07, abs=1e-14)
    assert s["y"][0] == 0.0 and s["vy"][1] == 0.0


def test_head_on_perfectly_inelastic_f1(orc):
    """f = 1: the normal relative velocity vanishes after the impact (both move with the
    centre-of-mass velocity along the line of centres)."""
    m1, m2 = 2e-6, 1e-6
    s = _state([(-0.05, 0, 0, 1.0, 0, 0, m1, 0.01), (0.05, 0, 0, -1.0, 0, 0, m2, 0.01)])
    orc.resolve(s, [[0, 1]], 0.1, 1.0)
    vcm = (m1 * 1.0 + m2 * -1.0) / (m1 + m2)
    assert s["vx"][0] == pytest.approx(vcm, abs=1e-14)
    assert s["vx"][1] == pytest.approx(vcm, abs=1e-14)


def _colliding_pairs(orc, d, dt):
    pairs = orc.pairs_brute(d, dt)
    assert len(pairs) > 20
    return pairs


@pytest.mark.parametrize("f", [1.0, 1.3, 2.0])
def test_conservation_and_energy_change(orc, f):
    """Momentum is conserved by every impulse; the kinetic energy changes by
    alpha s^2 (alpha (R1+R2)^2 (m1+m2)/(2 m1 m2) - 1) per resolved pair (Sect. 5.1),
    i.e. not at all for f = 2; the normal relative velocity becomes (1 - f) times its
    value before the impact (Sect. 5.2)."""
    d = inputs.gas_box(2000, seed=3, radius=0.01)
    d["m"] = d["m"] * (1.0 + np.arange(2000) % 7)          # unequal masses
    dt = 0.01
    pairs = _colliding_pairs(orc, d, dt)
    s = {k: v.copy() for k, v in d.items()}
    res = orc.resolve(s, pairs, dt, f)
    assert len(res) > 10
    p0 = np.array([(d["m"] * d[v]).sum() for v in ("vx", "vy", "vz")])
    p1 = np.array([(s["m"] * s[v]).sum() for v in ("vx", "vy", "vz")])
    scale = (d["m"] * np.abs(d["vx"])).sum()
    assert np.abs(p1 - p0).max() <= 1e-14 * scale
    ke = lambda st: 0.5 * (st["m"] * (st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2)).sum()
    want = 0.0
    for i, j in res:
        t = orc.collision_time((d["x"][i], d["y"][i], d["z"][i]),
                               (d["vx"][i], d["vy"][i], d["vz"][i]), d["R"][i],
                               (d["x"][j], d["y"][j], d["z"][j]),
                               (d["vx"][j], d["vy"][j], d["vz"][j]), d["R"][j], dt)
        r = np.array([d[a][i] - d[a][j] for a in ("x", "y", "z")])
        v = np.array([d[a][i] - d[a][j] for a in ("vx", "vy", "vz")])
        dr = r + t * v
        Rs = d["R"][i] + d["R"][j]
        # contact: the straight lines bring the spheres exactly into touch at dt_c
        assert np.linalg.norm(dr) == pytest.approx(Rs, rel=1e-9)
        m1, m2 = d["m"][i], d["m"][j]
        alpha = f * m1 * m2 / ((m1 + m2) * Rs * Rs)
        sdot = dr @ v
        want += alpha * sdot ** 2 * (alpha * Rs ** 2 * (m1 + m2) / (2 * m1 * m2) - 1.0)
        # normal relative velocity after the impact
        v_after = np.array([s[a][i] - s[a][j] for a in ("vx", "vy", "vz")])
        assert dr @ v_after == pytest.approx((1.0 - f) * sdot, rel=1e-9, abs=1e-12 * abs(sdot))
    got = ke(s) - ke(d)
    assert got == pytest.approx(want, rel=1e-9, abs=1e-15 * ke(d))
    if f == 2.0:
        assert abs(got) <= 1e-13 * ke(d)


def test_greedy_takes_earliest_contact(orc):
    """A moonlet collides at most once per step; the earliest contact wins."""
    R = 0.01
    # 0 meets 1 at t = 0.01; 1 would meet 2 at t = 0.02 -> only (0, 1)
    s = _state([(-0.04, 0, 0, 1.0, 0, 0, 1e-6, R), (0.0, 0, 0, 0.0, 0, 0, 1e-6, R),
                (0.06, 0, 0, -1.0, 0, 0, 1e-6, R)])
    res = orc.resolve(s, [[0, 1], [1, 2]], 0.1, 2.0)
    assert res.tolist() == [[0, 1]]
    # the middle pair is first: both outer pairs are dropped
    s = _state([(-0.2, 0, 0, 1.0, 0, 0, 1e-6, R), (0.0, 0, 0, 0.2, 0, 0, 1e-6, R),
                (0.03, 0, 0, -0.2, 0, 0, 1e-6, R), (0.3, 0, 0, -1.0, 0, 0, 1e-6, R)])
    res = orc.resolve(s, [[0, 1], [1, 2], [2, 3]], 0.5, 2.0)
    assert res.tolist() == [[1, 2]]


def test_greedy_matching_properties(orc):
    """On a dense gas box: the resolved pairs form a matching, and every pair left out
    shares a moonlet with a resolved pair of earlier (dt_c, i, j) -- which is exactly
    the greedy rule, checked here without re-running it."""
    d = inputs.gas_box(3000, seed=5, radius=0.015)
    dt = 0.02
    pairs = _colliding_pairs(orc, d, dt)
    s = {k: v.copy() for k, v in d.items()}
    res = orc.resolve(s, pairs, dt, 1.5)
    used = {}
    key = {}
    for i, j in pairs:
        t = orc.collision_time((d["x"][i], d["y"][i], d["z"][i]),
                               (d["vx"][i], d["vy"][i], d["vz"][i]), d["R"][i],
                               (d["x"][j], d["y"][j], d["z"][j]),
                               (d["vx"][j], d["vy"][j], d["vz"][j]), d["R"][j], dt)
        key[(i, j)] = (t, i, j)
    for i, j in res:
        assert i not in used and j not in used
        used[i] = used[j] = key[(i, j)]
    resolved = set(map(tuple, res.tolist()))
    assert len(resolved) < len(pairs)        # some moonlets had several partners
    for i, j in pairs:
        if (i, j) in resolved:
            continue
        blockers = [used[k] for k in (i, j) if k in used]
        assert blockers and min(blockers) < key[(i, j)]
    # every resolved pair is unblocked by any earlier resolved pair
    for i, j in res:
        assert used[i] == used[j] == key[(i, j)]

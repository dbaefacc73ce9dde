"""Pins for the oracle's pair test (Sect. 3.1, Eqs. 1-2), the collision climb and
walk (Eqs. 7-9, Alg. 2), and the leapfrog (Sect. 4.1)."""
import math

import numpy as np
import pytest

from paper_2310_20374_amd import inputs


def test_head_on_closed_form(orc):
    """Moonlet 1 at the origin moving at u towards moonlet 2 at distance d: contact
    after (d - R1 - R2)/u exactly."""
    d, u, R1, R2 = 1.0, 2.0, 0.125, 0.25
    tc = (d - R1 - R2) / u           # 0.3125, exact in binary
    r1, v1 = (0.0, 0.0, 0.0), (u, 0.0, 0.0)
    r2, v2 = (d, 0.0, 0.0), (0.0, 0.0, 0.0)
    assert orc.pair_test(r1, v1, R1, r2, v2, R2, tc)            # contact at dt: included
    assert orc.pair_test(r1, v1, R1, r2, v2, R2, 0.5)
    assert not orc.pair_test(r1, v1, R1, r2, v2, R2, 0.3)
    # symmetric in the two moonlets
    assert orc.pair_test(r2, v2, R2, r1, v1, R1, tc)


def test_pair_test_negative_cases(orc):
    R = 0.1
    # receding: contact happened in the past
    assert not orc.pair_test((0, 0, 0), (-1, 0, 0), R, (1, 0, 0), (0, 0, 0), R, 10.0)
    # no relative motion (dv^2 = 0): never, even when touching
    assert not orc.pair_test((0, 0, 0), (1, 1, 0), R, (0.15, 0, 0), (1, 1, 0), R, 1.0)
    # miss: impact parameter above R1 + R2, Delta < 0
    assert not orc.pair_test((0, 0, 0), (1, 0, 0), R, (2, 0.25, 0), (0, 0, 0), R, 10.0)
    # grazing within the sum of radii: hits
    assert orc.pair_test((0, 0, 0), (1, 0, 0), R, (2, 0.15, 0), (0, 0, 0), R, 10.0)
    # already overlapping and approaching: Delta t < 0 by Eq. (2), not counted
    assert not orc.pair_test((0, 0, 0), (1, 0, 0), R, (0.1, 0, 0), (0, 0, 0), R, 1.0)


def test_gas_box_rate(orc):
    """Collision count of a dilute gas of spheres against kinetic theory,
    N(N-1)/2 pi S^2 <|dv|> dt / V, averaged over seeds (Poisson tolerance)."""
    n, R, sig, dt = 2000, 0.01, 1.0, 0.01
    exp = inputs.gas_box_expected_pairs(n, R, sig, dt)
    counts = []
    for seed in range(5):
        d = inputs.gas_box(n, seed=seed, radius=R, sigma=sig)
        counts.append(len(orc.pairs_brute(d, dt)))
    mean = np.mean(counts)
    # edge effects of the finite box reduce the rate a little
    assert abs(mean - exp) < 4 * math.sqrt(exp / 5) + 0.1 * exp, (counts, exp)


@pytest.mark.parametrize("case", ["gas", "disk_big_dt", "hot", "clumps"])
def test_tree_pairs_equal_brute_force(orc, case):
    """Well-separated cells cannot collide (Sect. 3.4.3), so the walk finds
    exactly the brute-force pair set."""
    if case == "gas":
        d, dt, s = inputs.gas_box(2000, seed=1), 0.01, 8
    elif case == "disk_big_dt":
        d, dt, s = inputs.disk(3000, seed=2), 2.0, 16
    elif case == "hot":
        d, dt, s = inputs.hot_disk(3000, seed=0), 0.5, 17
    else:
        d, dt, s = inputs.clumps(4000, seed=0, n_clumps=10), 0.01, 16
    ref = orc.pairs_brute(d, dt)
    t = orc.Tree(d["x"], d["y"], d["z"], s)
    c = orc.Collide(t, d["vx"], d["vy"], d["vz"], d["R"], dt)
    got = c.run(12, 0, 16)
    assert len(ref) > 0 or case == "disk_big_dt"
    assert np.array_equal(got, ref)
    # the walk tested far fewer pairs than brute force
    n = len(d["x"])
    assert c.ntests() < n * (n - 1) // 2


@pytest.mark.parametrize("case", ["gas", "disk_big_dt", "hot", "clumps", "clumps_1e5",
                                  "coincident", "static"])
def test_grid_pairs_equal_brute_force(orc, case):
    """The grid-filtered scan (the exact pair oracle for inputs too large for the
    all-pairs scan) returns exactly the all-pairs set of Eqs. (1)-(2): a pair that
    touches within dt started at most R_i + R_j + dt(|v_i| + |v_j|) apart, so it sits
    in the same or adjacent grid cells."""
    if case == "gas":
        d, dt = inputs.gas_box(2000, seed=3), 0.01
    elif case == "disk_big_dt":
        d, dt = inputs.disk(20000, seed=4), 1.0
    elif case == "hot":
        d, dt = inputs.hot_disk(20000, seed=5), 3.0
    elif case == "clumps":
        d, dt = inputs.clumps(20000, seed=6, n_clumps=10), 0.01
    elif case == "clumps_1e5":
        d, dt = inputs.clumps(100000, seed=7, n_clumps=50), 1e-3
    elif case == "coincident":
        d, dt = inputs.coincident(3000, seed=8), 0.3
    else:
        # nothing moves: only pairs already overlapping, and Eq. (2) rejects those
        d, dt = inputs.gas_box(2000, seed=9, radius=0.02), 0.1
        for k in ("vx", "vy", "vz"):
            d[k] = np.zeros_like(d[k])
    want = orc.pairs_brute(d, dt)
    got = orc.pairs_grid(d, dt)
    assert np.array_equal(got, want)
    if case in ("gas", "disk_big_dt", "hot", "clumps", "clumps_1e5"):
        assert len(want) > 20
    if case == "static":
        assert len(want) == 0


def test_grid_pairs_catch_reach_at_the_cell_edge(orc):
    """Two moonlets heading at each other from just under the largest possible
    separation R1 + R2 + dt (|v1| + |v2|) collide exactly at dt; the grid scan must
    still list them (the cells are sized from the largest reach)."""
    R, u, dt = 0.01, 0.5, 0.2
    sep = 2 * R + 2 * u * dt * (1 - 1e-9)
    for shift in (0.0, 0.37, -1.91):
        d = {"x": np.array([shift, shift + sep, 5.0]), "y": np.zeros(3), "z": np.zeros(3),
             "vx": np.array([u, -u, 0.0]), "vy": np.zeros(3), "vz": np.zeros(3),
             "R": np.array([R, R, R])}
        assert orc.pairs_brute(d, dt).tolist() == [[0, 1]]
        assert orc.pairs_grid(d, dt).tolist() == [[0, 1]]


def test_collision_climb_bounds(orc):
    """r_max bounds every moonlet's distance from the centre and r_crit - r_max
    bounds R + dt |v| of every moonlet (Eqs. 8-9 by induction)."""
    d = inputs.clumps(3000, seed=1, n_clumps=8)
    dt = 0.05
    t = orc.Tree(d["x"], d["y"], d["z"], 10)
    c = orc.Collide(t, d["vx"], d["vy"], d["vz"], d["R"], dt)
    cells = c.cells()
    P = np.stack([d["x"], d["y"], d["z"]], 1)[t.perm]
    V = np.stack([d["vx"], d["vy"], d["vz"]], 1)[t.perm]
    Rr = d["R"][t.perm]
    for k in range(t.ncells):
        sl = slice(t.first[k], t.first[k] + t.count[k])
        dist = np.linalg.norm(P[sl] - cells["sbar"][k], axis=1)
        assert dist.max() <= cells["rmax"][k] * (1 + 1e-12)
        ext = (Rr[sl] + dt * np.linalg.norm(V[sl], axis=1)).max()
        assert ext <= (cells["rcrit"][k] - cells["rmax"][k]) * (1 + 1e-12)
        assert np.allclose(cells["sbar"][k], P[sl].mean(0), rtol=1e-12, atol=1e-13)


def test_kepler_leapfrog_second_order(orc):
    """A single moonlet (no mutual gravity): the merged kick-drift-kick of
    Sect. 4.1 keeps the Kepler energy bounded with an O(dt^2) error."""
    d = {"x": np.array([3.0]), "y": np.array([0.0]), "z": np.array([0.0]),
         "vx": np.array([0.0]), "vy": np.array([math.sqrt(1 / 3.0) * 1.1]),
         "vz": np.array([0.0]), "m": np.array([1e-9]), "R": np.array([0.01])}

    def energy(s):
        return 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2) - \
            1.0 / np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2)

    E0 = energy(d)[0]
    period = 2 * math.pi * (1.0 / (2 / 3.0 - (1 / 3.0) * 1.21)) ** 1.5
    errs = []
    for k in (400, 800):
        dt = period / k
        s, worst = d, 0.0
        for _ in range(8):                      # error envelope over one orbit
            s, _ = orc.kdk_steps(s, dt, k // 8, None)
            worst = max(worst, abs(energy(s)[0] - E0))
        errs.append(worst)
        # returns to the start after one period to O(dt^2)
        assert abs(s["x"][0] - 3.0) < 50 * dt * dt
    assert 3.0 < errs[0] / errs[1] < 5.0
    assert errs[0] < 1e-3 * abs(E0)

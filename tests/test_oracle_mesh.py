"""Pins of the oracle's mesh module (Sect. 3.3): the paper's worked numbers for
Eqs. (4)-(5), the neighbourhood on hand-placed moonlets, the neighbour count of a
lattice in closed form, Eq. (6), the limits where the mesh reduces to the direct
sum and to brute-force collision search, and the role of the three most massive
and of the oversized moonlets."""
import numpy as np
import pytest

from paper_2310_20374_amd import inputs

R_EARTH_KM = 6371.0
R_MOON_KM = 1737.4


def test_worked_example_gamma(orc):
    """h/r = 0.05, R_max = 10 R_Earth, N = 1e5, x = 8: gamma = 0.08526 R_Earth, i.e.
    543.2 km (Sect. 3.3)."""
    g = orc.mesh_gamma_crit(8, 1e5, 0.05, 10.0)
    assert round(g, 5) == 0.08526
    assert round(g * R_EARTH_KM, 1) == 543.2


def test_worked_example_radius_and_aspect(orc):
    """One Moon mass in 1e5 moonlets: mean radius 37.4 km, which fits the mesh
    (2R <= gamma); Eq. (5) asks h/r >= 1.307e-4 for x = 8, R_max = 10 R_Earth."""
    R = R_MOON_KM / 1e5 ** (1 / 3)
    assert round(R, 1) == 37.4
    assert 2 * R <= orc.mesh_gamma_crit(8, 1e5, 0.05, 10.0) * R_EARTH_KM
    a = orc.mesh_aspect_crit(8, R_MOON_KM / (10 * R_EARTH_KM))
    assert round(a * 1e4, 3) == 1.307
    # at exactly that aspect ratio the critical mesh is the moonlets' diameter: Eq. (5)
    # is Eq. (4) solved for 2R = gamma with N = (R_Moon / R)^3
    N = 1e5
    g = orc.mesh_gamma_crit(8, N, a, 10.0 * R_EARTH_KM)
    R = R_MOON_KM / N ** (1 / 3)
    s = a * a / (1 + a * a)
    assert g / (2 * R) == pytest.approx((s / (a * a)) ** (1 / 6), rel=1e-12)


def _pts(rows, R=0.01, m=None):
    a = np.array(rows, dtype=np.float64)
    n = len(a)
    z = np.zeros(n)
    return {"x": a[:, 0], "y": a[:, 1], "z": a[:, 2], "vx": z.copy(), "vy": z.copy(),
            "vz": z.copy(), "m": np.full(n, 1e-6) if m is None else np.asarray(m, float),
            "R": np.full(n, R)}


def test_neighbourhood_by_hand(orc):
    """gamma = 1: cells are unit cubes with floor; a moonlet's neighbourhood is the
    3 x 3 x 3 block around its cell, across the origin too."""
    d = _pts([(0.5, 0.5, 0.5), (1.5, 1.5, 1.5), (2.5, 0.5, 0.5), (-0.5, 0.5, 0.5),
              (-1.5, 0.5, 0.5), (0.5, -0.99, 1.99)])
    # cells: (0,0,0) (1,1,1) (2,0,0) (-1,0,0) (-2,0,0) (0,-1,1)
    # adjacent: 0-1, 0-3 (across the origin), 0-5, 1-2, 3-4, 3-5;
    # not: 0-2, 0-4, 1-3, 1-5 (dy 2), 2-5, 4-5, ... (some offset of 2)
    pairs = {(0, 1), (0, 3), (0, 5), (1, 2), (3, 4), (3, 5)}
    # moonlets 3, 4, 5 are the most massive: they feel, and act on, everyone
    d["m"] = np.array([1e-6, 2e-6, 3e-6, 4e-6, 5e-6, 6e-6])
    flags = orc.mesh_flags(d["m"], d["R"], 1.0)
    assert flags.tolist() == [0, 0, 0, 2, 2, 2]
    a = orc.mesh_accel(d, 1.0)
    big = {3, 4, 5}
    n = 6
    want = np.zeros((n, 3))
    pos = np.stack([d["x"], d["y"], d["z"]], 1)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            if i in big or j in big or (min(i, j), max(i, j)) in pairs:
                r = pos[j] - pos[i]
                want[i] += d["m"][j] * r / np.linalg.norm(r) ** 3
    assert np.allclose(a, want, rtol=1e-14, atol=0)
    # x': mesh neighbours counted over all moonlets of the mesh (the big ones too)
    assert orc.mesh_neighbours(d, 1.0) == pytest.approx(2 * len(pairs) / n, abs=0)


@pytest.mark.parametrize("k", [1, 2, 5])
def test_lattice_neighbour_count(orc, k):
    """One moonlet at the centre of each cell of a k x k x k block: the mean number of
    neighbours is ((3k - 2)/k)^3 - 1 (26 in the interior)."""
    g = 0.1
    c = (np.arange(k) + 0.5) * g - 0.37       # shifted off the origin
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    d = _pts(np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1), R=0.01)
    want = ((3 * k - 2) / k) ** 3 - 1
    assert orc.mesh_neighbours(d, g) == pytest.approx(want, rel=1e-14)


def test_gamma_update_eq6(orc):
    """Eq. (6): gamma' (x/x')^(1/3); the clamp at gamma_min; x' = 0 doubles."""
    assert orc.mesh_gamma_next(0.2, 8.0, 1.0) == pytest.approx(0.4, rel=1e-15)
    assert orc.mesh_gamma_next(0.2, 8.0, 27.0) == pytest.approx(0.2 * 2 / 3, rel=1e-15)
    assert orc.mesh_gamma_next(0.2, 8.0, 64.0, gamma_min=0.15) == 0.15
    assert orc.mesh_gamma_next(0.2, 8.0, 0.0) == 0.4
    # the update drives the lattice towards the target count: cells of a uniform
    # cloud hold gamma^3 n moonlets, so one update lands near x
    rng = np.random.default_rng(3)
    n = 20000
    d = _pts(rng.random((n, 3)), R=1e-5)
    g0 = 0.05
    x1 = orc.mesh_neighbours(d, g0)
    g1 = orc.mesh_gamma_next(g0, 8.0, x1)
    assert orc.mesh_neighbours(d, g1) == pytest.approx(8.0, rel=0.15)


def test_one_cell_is_direct_sum(orc):
    """A mesh larger than the system: every pair interacts, gravity is the direct sum
    and the collision pairs are the brute-force pairs."""
    d = inputs.gas_box(1500, seed=4, radius=0.01)
    g = 100.0
    a = orc.mesh_accel(d, g)
    ex = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    assert np.abs(a - ex).max() <= 1e-13 * np.abs(ex).max()
    assert np.array_equal(orc.mesh_pairs(d, g, 0.01), orc.pairs_brute(d, 0.01))


def test_fine_mesh_finds_every_collision(orc):
    """Moonlets no larger than the mesh that move less than a cell per step: every
    colliding pair lies in adjacent cells, so the mesh finds the brute-force pairs."""
    d = inputs.gas_box(3000, seed=5, radius=0.01)
    dt = 0.005
    g = 0.1
    assert np.all(2 * d["R"] <= g)
    vmax = np.sqrt(d["vx"] ** 2 + d["vy"] ** 2 + d["vz"] ** 2).max()
    assert 2 * d["R"].max() + 2 * vmax * dt <= g
    want = orc.pairs_brute(d, dt)
    assert len(want) > 10
    assert np.array_equal(orc.mesh_pairs(d, g, dt), want)
    # a mesh finer than the pair distances misses some
    assert len(orc.mesh_pairs(d, 0.021, dt)) < len(want)


def test_mesh_gravity_misses_far_pairs_but_keeps_the_big_three(orc):
    """With a fine mesh, gravity is exact for a moonlet's neighbours and the three most
    massive moonlets only: removing every other moonlet leaves a moonlet's
    acceleration unchanged."""
    d = inputs.disk(800, seed=6)
    d["m"][[5, 300, 700]] *= 1000.0
    g = 0.3
    a = orc.mesh_accel(d, g)
    fl = orc.mesh_flags(d["m"], d["R"], g)
    assert sorted(np.nonzero(fl & 2)[0].tolist()) == [5, 300, 700]
    cell = np.floor(np.stack([d["x"], d["y"], d["z"]], 1) / g).astype(np.int64)
    for i in (0, 123, 456, 5):
        if fl[i]:
            keep = np.arange(len(d["x"]))       # a big one feels everyone
        else:
            adj = np.all(np.abs(cell - cell[i]) <= 1, axis=1)
            keep = np.nonzero(adj | (fl != 0))[0]
        sub = {k: v[keep] for k, v in d.items()}
        ex = orc.direct_sum(sub["x"], sub["y"], sub["z"], sub["m"])
        ii = int(np.nonzero(keep == i)[0][0])
        assert np.allclose(a[i], ex[ii], rtol=1e-13, atol=0), i
    # and the mutual sum is not the full one
    full = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    rel = np.linalg.norm(a - full, axis=1) / np.linalg.norm(full, axis=1)
    assert np.median(rel) > 0.01


def test_oversized_moonlet_interacts_with_all(orc):
    """A moonlet with 2R > gamma is kept out of the mesh and tested against every
    other moonlet for collisions; moonlets of the mesh collide only with neighbours."""
    d = _pts([(0.05, 0.05, 0.05), (0.9, 0.05, 0.05), (0.5, 0.05, 0.05)], R=0.01)
    d["vx"] = np.array([3.0, -10.0, 0.0])
    d["R"] = np.array([0.01, 0.01, 0.3])     # moonlet 2 is oversized for gamma = 0.25
    dt = 0.1
    g = 0.25
    fl = orc.mesh_flags(d["m"], d["R"], g)
    assert fl[2] & 1
    # all three pairs meet within dt; 0 (cell 0) and 1 (cell 3) are not neighbours
    assert orc.pairs_brute(d, dt).tolist() == [[0, 1], [0, 2], [1, 2]]
    assert orc.mesh_pairs(d, g, dt).tolist() == [[0, 2], [1, 2]]
    # x' counts the mesh moonlets only: 0 and 1 have no neighbour
    assert orc.mesh_neighbours(d, g) == 0.0


def test_mesh_clock_follows_eq4_then_eq6(orc):
    d = inputs.disk(3000, seed=7)
    clk = orc.MeshClock(8.0, 0.05, gamma_min=0.0)
    clk.accel(d)
    rmax = np.sqrt(d["x"] ** 2 + d["y"] ** 2 + d["z"] ** 2).max()
    g0, x0 = clk.history[0]
    assert g0 == orc.mesh_gamma_crit(8.0, 3000, 0.05, rmax)
    clk.accel(d)
    g1, x1 = clk.history[1]
    assert g1 == orc.mesh_gamma_next(g0, 8.0, x0)
    assert abs(x1 - 8.0) < abs(x0 - 8.0)


def test_three_most_massive_ties_and_small_n(orc):
    """Equal masses: the smaller indices win; fewer than three moonlets: all of them."""
    m = np.array([1.0, 3.0, 2.0, 3.0, 3.0, 0.5])
    R = np.full(6, 1e-3)
    assert orc.mesh_flags(m, R, 1.0).tolist() == [0, 2, 0, 2, 2, 0]
    m = np.full(5, 1.0)
    assert orc.mesh_flags(m, np.full(5, 1e-3), 1.0).tolist() == [2, 2, 2, 0, 0]
    assert orc.mesh_flags(np.array([1.0, 2.0]), np.full(2, 1e-3), 1.0).tolist() == [2, 2]


def test_sampled_forms_equal_full_forms(orc):
    """Per-target accelerations and pairs equal the full results restricted to them."""
    d = inputs.gas_box(3000, seed=13, radius=0.01)
    d["R"][[3, 30]] = 0.08                      # two oversized moonlets for gamma = 0.1
    tg = np.arange(0, 3000, 7)
    assert np.array_equal(orc.mesh_accel_of(d, 0.1, tg), orc.mesh_accel(d, 0.1)[tg])
    allp = orc.mesh_pairs(d, 0.1, 0.005)
    want = allp[np.isin(allp[:, 0], tg) | np.isin(allp[:, 1], tg)]
    assert len(want) > 5
    assert np.array_equal(orc.mesh_pairs_of(d, 0.1, 0.005, tg), want)

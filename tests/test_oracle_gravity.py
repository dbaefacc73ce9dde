"""Pins for the oracle's gravity: derivative tensors (Eq. 17), multipoles
(Eq. 20), interaction tensors (Eq. 25), the shift (Eq. 26), the mass-dependent
opening angle (recalled from Dehnen 2002) and the complete falcON walk (Alg. 2) against closed forms, invariants
and the paper's printed accuracy."""
import json
import math
import os

import numpy as np
import pytest

from paper_2310_20374_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _errs(a, ref):
    e = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return float(np.sqrt(np.mean(e * e))), float(e.max())


# --------------------------------------------------------------- Eq. (17)
@pytest.mark.parametrize("n", range(0, 7))
def test_green_derivs_along_axis(orc, n):
    """d^n/dx^n (1/x) = (-1)^n n! / x^(n+1) on the x-axis."""
    x = 1.7
    D = orc.green_derivs(np.array([x, 0.0, 0.0]), 6)
    assert D[n, 0, 0] == pytest.approx((-1) ** n * math.factorial(n) / x ** (n + 1), rel=1e-13)


def test_green_derivs_traceless_and_symmetric(orc):
    R = np.array([0.7, -1.3, 0.4])
    for n in range(2, 7):
        F = orc.green_deriv_full(R, n)
        # symmetric under any swap of two indices
        for a in range(n):
            for b in range(a + 1, n):
                assert np.allclose(F, np.swapaxes(F, a, b), rtol=0, atol=1e-12 * np.abs(F).max())
        # Laplace: contracting any index pair gives zero
        tr = np.trace(F, axis1=0, axis2=1)
        assert np.abs(tr).max() < 1e-11 * np.abs(F).max()


def test_green_derivs_finite_differences(orc):
    R = np.array([1.1, 0.6, -0.8])
    h = 1e-5
    for n in range(1, 7):
        F = orc.green_deriv_full(R, n)
        for k in range(3):
            e = np.zeros(3); e[k] = h
            Fp = orc.green_deriv_full(R + e, n - 1)
            Fm = orc.green_deriv_full(R - e, n - 1)
            fd = (Fp - Fm) / (2 * h)
            # last index of F is the newest derivative (Eq. 17)
            assert np.allclose(F[..., k], fd, rtol=1e-6, atol=1e-7 * np.abs(F).max())


def test_green_derivs_odd_under_reflection(orc):
    R = np.array([0.9, 0.2, -1.4])
    for n in range(0, 7):
        assert np.allclose(orc.green_deriv_full(-R, n), (-1) ** n * orc.green_deriv_full(R, n),
                           rtol=1e-13, atol=0)


# --------------------------------------------------------------- Eq. (20)
def test_multipoles_two_masses(orc):
    """Two equal masses at +-d e_x about the centre: M^(2)_xx = 2 mu d^2, every
    other quadrupole component 0, M^(0) = 2 mu (App. C: M^(1) vanishes)."""
    d, mu = 0.3, 0.25
    x = np.array([-d, d]); y = np.zeros(2); z = np.zeros(2)
    t = orc.Tree(x, y, z, 4)                 # root is a leaf
    g = orc.Gravity(t, np.full(2, mu), 1.0, 4, 0.5, 1)
    M, _ = g.cell_tensors(0)
    M0, M2, M3 = M[0], M[1:10].reshape(3, 3), M[10:37].reshape(3, 3, 3)
    assert M0 == pytest.approx(2 * mu)
    ref = np.zeros((3, 3)); ref[0, 0] = 2 * mu * d * d
    assert np.allclose(M2, ref, atol=1e-16)
    assert np.allclose(M3, 0.0, atol=1e-16)
    c = g.cells()
    assert np.allclose(c["s"][0], 0.0, atol=1e-16) and c["mass"][0] == pytest.approx(2 * mu)


def test_multipole_translation_is_binomial(orc):
    """The parent's moments equal the children's moments shifted binomially
    (App. C); checked on a random tree against moments of the children."""
    d = inputs.disk(800, seed=4)
    t = orc.Tree(d["x"], d["y"], d["z"], 20)
    g = orc.Gravity(t, d["m"], 1.0, 6, 0.5)
    cells = g.cells()
    c = int(np.where(t.nchild > 1)[0][-1])
    Mp, _ = g.cell_tensors(c)
    acc = np.zeros_like(Mp)
    for ch in range(t.child_first[c], t.child_first[c] + t.nchild[c]):
        Mc, _ = g.cell_tensors(ch)
        lam = cells["s"][c] - cells["s"][ch]          # Lambda = s_B - s_b
        blocks_c = {0: Mc[0:1], 2: Mc[1:10], 3: Mc[10:37], 4: Mc[37:118], 5: Mc[118:361]}
        # sum_k binom(n,k) (-Lambda)^(k) (x) m^(n-k), symmetrised by full expansion
        out = []
        for n in (0, 2, 3, 4, 5):
            T = np.zeros((3,) * n) if n else np.zeros(())
            for k in range(0, n + 1):
                if n - k == 1:
                    continue
                mk = blocks_c[n - k].reshape((3,) * (n - k)) if n - k else blocks_c[0][0]
                lk = np.ones(())
                for _ in range(k):
                    lk = np.multiply.outer(lk, -lam)
                outer = np.multiply.outer(lk, mk)
                # symmetrise over all index orders
                import itertools
                perms = list(itertools.permutations(range(n))) if n else [()]
                sym = sum(np.transpose(outer, p) for p in perms) / len(perms) if n else outer
                T = T + math.comb(n, k) * sym
            out.append(np.ravel(T))
        acc += np.concatenate(out)
    assert np.allclose(acc, Mp, rtol=1e-9, atol=1e-12 * np.abs(Mp).max())


# --------------------------------------------------------------- Eq. (25)-(26)
def test_single_cell_pair_converges_geometrically(orc):
    """A source cluster seen from a target cluster: the expansion error falls like
    ((r_A + r_B)/R)^(p+1) (remainder of Eq. 25)."""
    rng = np.random.default_rng(1)
    src = rng.normal(size=(20, 3)) * 0.1
    mu = rng.uniform(0.5, 1.0, 20)
    tgt = rng.normal(size=(10, 3)) * 0.1 + np.array([2.0, 0.5, 0.3])
    sA = tgt.mean(0)
    exact = np.zeros((10, 3))
    for i in range(10):
        dd = src - tgt[i]
        r = np.linalg.norm(dd, axis=1)
        exact[i] = (mu[:, None] * dd / r[:, None] ** 3).sum(0)
    prev = None
    for p in range(1, 7):
        a = orc.expansion_field(src, mu, sA, tgt, p)
        err = np.abs(a - exact).max() / np.abs(exact).max()
        if prev is not None:
            assert err < 0.35 * prev, (p, err, prev)
        prev = err
    assert prev < 1e-4


def test_shift_is_exact_reexpansion(orc):
    """Eq. (26) moves a degree-p local expansion without changing it: evaluating
    after the shift equals evaluating before."""
    rng = np.random.default_rng(7)
    p = 6
    import itertools
    blocks = []
    for m in range(1, p + 1):
        T = rng.normal(size=(3,) * m)
        perms = list(itertools.permutations(range(m)))
        T = sum(np.transpose(T, q) for q in perms) / len(perms)
        blocks.append(T.ravel())
    Cin = np.concatenate(blocks)
    d = np.array([0.13, -0.07, 0.05])
    Cout = orc.shift_C(Cin, p, d)

    def accel(Cflat, delta):
        off, acc = 0, np.zeros(3)
        Cs = []
        for m in range(1, p + 1):
            Cs.append(Cflat[off:off + 3 ** m].reshape((3,) * m)); off += 3 ** m
        for n in range(0, p):
            T = Cs[n]
            for _ in range(n):
                T = T @ delta
            acc += T / math.factorial(n)
        return acc

    x = np.array([0.02, 0.04, -0.03])
    assert np.allclose(accel(Cout, x), accel(Cin, x + d), rtol=1e-12, atol=1e-12)


# ------------------------------------------------- mass-dependent opening angle
def test_theta_of_mass(orc):
    """Self-consistency of the bisection only (the relation is recalled from Dehnen
    2002, not printed in the paper); what pins
    theta(M) to the paper is the Fig. 4 accuracy test below."""
    tmin = 0.5
    assert orc.theta_of_mass(1.0, 1.0, tmin) == tmin
    prev = tmin
    K = tmin ** 5 / (1 - tmin) ** 2
    for ratio in (0.5, 1e-1, 1e-2, 1e-4, 1e-6):
        th = orc.theta_of_mass(ratio, 1.0, tmin)
        assert tmin < th < 1.0 and th > prev
        prev = th
        lhs = th ** 5 / (1 - th) ** 2
        assert lhs == pytest.approx(K * ratio ** (-1.0 / 3.0), rel=1e-12)


# --------------------------------------------------------------- whole walk
def test_no_opening_gives_direct_sum(orc):
    """N <= N_cs: the root self-interaction is brute force (Alg. 2)."""
    d = inputs.disk(1500, seed=3)
    ad = orc.direct_sum(d["x"], d["y"], d["z"], d["m"])
    a, t, g = orc.tree_accel(d, p=3, s=16, ncs=10 ** 9)
    assert g.counts()["m2l"] == 0
    assert _errs(a, ad)[1] < 1e-12


def test_two_body(orc):
    x = np.array([0.0, 3.0]); y = np.zeros(2); z = np.zeros(2); m = np.array([2.0, 0.5])
    G = 1.3
    a, _, _ = orc.tree_accel({"x": x, "y": y, "z": z, "m": m}, G=G, p=3, s=1, ncs=0, ncc_pre=0,
                             ncc_post=0)
    assert a[0, 0] == pytest.approx(G * 0.5 / 9.0, rel=1e-15)
    assert a[1, 0] == pytest.approx(-G * 2.0 / 9.0, rel=1e-15)
    assert np.all(a[:, 1:] == 0.0)


def test_p0_is_no_mutual_gravity(orc):
    d = inputs.disk(500, seed=0)
    a, _, _ = orc.tree_accel(d, p=0, s=16)
    assert np.all(a == 0.0)


@pytest.mark.parametrize("p", [1, 3, 6])
def test_momentum_conserved(orc, p):
    """Newton's third law holds to rounding for the falcON walk (Sect. 3.4.3)."""
    d = inputs.disk(4000, seed=5)
    a, _, g = orc.tree_accel(d, p=p, s=16, ncs=64, ncc_pre=8, ncc_post=64)
    assert g.counts()["m2l"] > 100
    f = d["m"][:, None] * a
    assert np.abs(f.sum(0)).max() < 1e-12 * np.abs(f).sum(0).max()


def test_tree_error_falls_geometrically_with_p(orc):
    """Two compact clusters: with constant theta the walk's interaction lists do
    not depend on p, and the error against the direct sum falls by a roughly
    constant factor per order (remainder of Eq. 25 ~ theta^(p+1))."""
    rng = np.random.default_rng(11)
    A = rng.normal(size=(200, 3)) * 0.05 + np.array([-4.0, 1.0, 0.0])
    B = rng.normal(size=(200, 3)) * 0.05 + np.array([5.0, -2.0, 0.5])
    P = np.concatenate([A, B])
    m = rng.uniform(0.5, 1.5, 400) * 1e-3
    d = {"x": P[:, 0], "y": P[:, 1], "z": P[:, 2], "m": m}
    ad = orc.direct_sum(d["x"], d["y"], d["z"], m)
    errs, lists = [], None
    for p in range(1, 7):
        a, t, g = orc.tree_accel(d, p=p, s=16, ncs=64, ncc_pre=8, ncc_post=64, theta_mode=1)
        c = g.counts()
        assert c["m2l"] >= 100
        lists = lists or c
        assert c == lists
        errs.append(_errs(a, ad)[0])
    ratios = np.array(errs[1:]) / np.array(errs[:-1])
    assert np.all(ratios < 0.6), errs
    assert errs[-1] < 2e-4


def test_uniform_sphere_field(orc):
    """Inside a uniform sphere of unit mass and radius the mean radial field is
    -G M(<r)/r^2 = -r (shell theorem); single-moonlet values scatter by the
    discreteness noise of an unsoftened field, so shells are averaged."""
    rng = np.random.default_rng(2)
    N = 20000
    u = rng.normal(size=(N, 3)); u /= np.linalg.norm(u, axis=1)[:, None]
    r = rng.uniform(0, 1, N) ** (1 / 3)
    P = u * r[:, None]
    m = np.full(N, 1.0 / N)
    d = {"x": P[:, 0], "y": P[:, 1], "z": P[:, 2], "m": m}
    a, _, _ = orc.tree_accel(d, p=4, s=16, ncs=64, ncc_pre=8, ncc_post=64)
    ar = (a * u).sum(1)
    for lo, hi in ((0.3, 0.5), (0.5, 0.7), (0.7, 0.85)):
        sel = (r > lo) & (r < hi)
        ratio = ar[sel] / (-r[sel])
        assert abs(ratio.mean() - 1.0) < 6 * ratio.std() / np.sqrt(sel.sum()) + 0.01
    # and the tree agrees with the direct sum far below that noise
    tg = np.arange(0, N, 97)
    ad = orc.direct_sum(d["x"], d["y"], d["z"], m, targets=tg)
    assert _errs(a[tg], ad)[0] < 1e-2


def _fig4_errors(orc, p, theta_mode, N=100_000, n_targets=2048):
    """Median of the paper's scalar relative error | |a| - |a_ref| | / |a_ref| on the
    Fig. 4 workload, for the mutual acceleration alone and with the central mass
    (the two families of curves of Fig. 4), at the leaf size and thresholds of the
    paper's runs at that order (Sect. 4.2)."""
    d = inputs.fig4_disk(N, seed=0)
    tg = inputs.sample_targets(N, n_targets)
    ad = orc.direct_sum(d["x"], d["y"], d["z"], d["m"], targets=tg)
    ac = orc.central_accel(d["x"][tg], d["y"][tg], d["z"][tg])
    s, thr = (17, (64, 8, 64)) if p <= 3 else (52, (256, 256, 512))
    a, _, _ = orc.tree_accel(d, p=p, s=s, ncs=thr[0], ncc_pre=thr[1], ncc_post=thr[2],
                             theta_mode=theta_mode)
    a = a[tg]

    def scalar(x, ref):
        return np.abs(np.linalg.norm(x, axis=1) - np.linalg.norm(ref, axis=1)) \
            / np.linalg.norm(ref, axis=1)
    return float(np.median(scalar(a, ad))), float(np.median(scalar(a + ac, ad + ac)))


@pytest.mark.slow
def test_fig4_accuracy_matches_paper(orc):
    """Sect. 4.2 with Fig. 4: at theta_min = 0.5 the relative acceleration error is of
    the order of 1e-5 at p = 3 and 1e-7 at p = 6, on 4e5 moonlets between 1 and 10
    Earth radii of total mass 0.024 (here 1e5 of them: the medians differ from 4e5 by
    about 10 %).  The printed magnitudes are those of the acceleration with the
    central mass (the mutual field alone of a disk is a residual of near-cancelling
    terms, and its relative error is ~10^2 larger).  Constant theta lands within 3x
    of both printed values; the mass-dependent angle, which the paper says it uses (its
    form recalled from Dehnen 2002), within 3x at p = 3 and about 5x at p = 6.  A wrong mass exponent in
    theta(M) (-1/2 instead of -1/3 doubles the opening of small cells) drives the
    p = 6 error above 1e-6 and fails here; so do a dropped expansion order or a
    wrong-signed term (errors of 1e-4 and up)."""
    gold = json.load(open(GOLDEN))["accuracy_theta_min_0.5"]
    res = {(p, mode): _fig4_errors(orc, p, mode) for p in (3, 6) for mode in (0, 1)}
    for (p, mode), (mut, tot) in res.items():
        print(f"p={p} theta_mode={mode}: median mutual {mut:.2e}, with central mass {tot:.2e}")
    # constant theta: within a factor 3 of the printed values at both orders
    assert gold["p3"] / 3 < res[(3, 1)][1] < 3 * gold["p3"]
    assert gold["p6"] / 3 < res[(6, 1)][1] < 3 * gold["p6"]
    # mass-dependent theta: 3x at p = 3; at p = 6 within 6x
    assert gold["p3"] / 3 < res[(3, 0)][1] < 3 * gold["p3"]
    assert gold["p6"] / 3 < res[(6, 0)][1] < 6 * gold["p6"]
    # the mass-dependent angle opens cells more widely, never less
    for p in (3, 6):
        assert res[(p, 0)][1] >= res[(p, 1)][1]
    # two orders of magnitude from p = 3 to p = 6 (printed: 1e-5 -> 1e-7)
    assert res[(3, 1)][1] / res[(6, 1)][1] > 30
    assert res[(3, 0)][1] / res[(6, 0)][1] > 20
    # the mutual-only error is far above the printed values (the other family)
    for key, (mut, tot) in res.items():
        assert mut > 20 * tot


def test_plummer_sphere_field(orc):
    """A Plummer sphere of mass M and scale b has the radial field
    -G M(<r)/r^2 with M(<r) = M r^3/(r^2 + b^2)^(3/2) (truncated at 10 b here, so the
    masses are those of the sphere inside 10 b).  The oracle tree, averaged over
    shells (an unsoftened field scatters by discreteness noise moonlet by moonlet),
    follows it from the core to the halo, and the direct sum does too."""
    N = 20000
    d = inputs.plummer_sphere(N, seed=3)
    P = np.stack([d["x"], d["y"], d["z"]], 1)
    r = np.linalg.norm(P, axis=1)
    u = P / r[:, None]
    inside_10b = 1000.0 / 101.0 ** 1.5            # M_P(<10 b) / M of the untruncated sphere
    field = -(r ** 3 / (r * r + 1.0) ** 1.5) / inside_10b / (r * r)
    a, _, _ = orc.tree_accel(d, p=4, s=16, ncs=64, ncc_pre=8, ncc_post=64)
    tg = np.arange(0, N, 7)
    ad = orc.direct_sum(d["x"], d["y"], d["z"], d["m"], targets=tg)
    ar = (a * u).sum(1)
    ard = (ad * u[tg]).sum(1)
    # the core's field follows the random realisation of its ~2000 moonlets (seeds
    # scatter by ~5 % there), the outer shells are set by many more
    for lo, hi, tol in ((0.2, 0.5, 0.12), (0.5, 1.0, 0.03), (1.0, 2.0, 0.02), (2.0, 4.0, 0.02)):
        sel = (r > lo) & (r < hi)
        assert abs(np.mean(ar[sel] / field[sel]) - 1.0) < tol, (lo, hi)
        seld = (r[tg] > lo) & (r[tg] < hi)
        assert abs(np.mean(ard[seld] / field[tg][seld]) - 1.0) < tol + 0.01, (lo, hi)
    # the tangential field averages to zero
    at = a - ar[:, None] * u
    assert np.abs(at.mean(0)).max() < 0.02 * np.abs(field).mean()
    assert _errs(a[tg], ad)[0] < 1e-2


def test_rmax_bounds_and_corner_clamp(orc):
    """r_max is an upper bound on every moonlet's distance from the expansion
    centre (Eq. 11) and never exceeds the distance to the farthest corner of the
    cell's cube (the clamp of Sect. 3.4.2); at a leaf it is exactly the smaller
    of the two."""
    d = inputs.clumps(3000, seed=2, n_clumps=6)
    t = orc.Tree(d["x"], d["y"], d["z"], 12)
    g = orc.Gravity(t, d["m"], 1.0, 4, 0.5)
    c = g.cells()
    P = np.stack([d["x"], d["y"], d["z"]], 1)[t.perm]
    L = t.L
    clamped = 0
    for k in range(t.ncells):
        sl = slice(t.first[k], t.first[k] + t.count[k])
        true_max = np.linalg.norm(P[sl] - c["s"][k], axis=1).max()
        assert true_max <= c["rmax"][k] * (1 + 1e-12)
        lev = int(t.level[k])
        q = np.array([orc.quantize(v, L) for v in P[t.first[k]]]) >> (21 - lev)
        h = L / 2 ** lev
        cen = -L + (2 * q + 1) * h
        corner = np.linalg.norm(np.abs(c["s"][k] - cen) + h)
        assert c["rmax"][k] <= corner * (1 + 1e-14)
        if t.nchild[k] == 0:
            assert c["rmax"][k] == pytest.approx(min(true_max, corner), rel=1e-14)
        clamped += c["rmax"][k] < corner * (1 - 1e-12)
    assert clamped > 0

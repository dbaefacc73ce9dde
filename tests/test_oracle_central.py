"""Pins of the oracle's central-body extras (App. B): the J2 bulge and the
quadrupolar tide of a distant body, against minus the gradient of the potentials
the paper gives (central finite differences), closed forms, and the exact
differential attraction of the distant body."""
import math

import numpy as np
import pytest

G, MC, J2, RC = 1.0, 1.0, 1.08e-3, 1.0
MS, AS, EPS = 332946.0, 23481.0, 0.4091


def _num_grad(V, p, h):
    g = np.zeros(3)
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g[k] = (V(p + e) - V(p - e)) / (2 * h)
    return g


def _acc(orc, p, **kw):
    return orc.central_accel(np.array([p[0]]), np.array([p[1]]), np.array([p[2]]), G, 0.0,
                             **kw)[0]


@pytest.mark.parametrize("p", [(3.0, 1.0, 0.5), (-2.0, 4.0, -1.5), (0.3, -0.2, 5.0)])
def test_j2_is_minus_gradient_of_its_potential(orc, p):
    p = np.array(p, dtype=np.float64)

    def V(q):                      # -G M R^2 J2 (r^2 - 3 z^2) / (2 r^5)
        r2 = q @ q
        return -G * MC * RC * RC * J2 * (r2 - 3 * q[2] ** 2) / (2 * r2 ** 2.5)

    want = -_num_grad(V, p, 1e-5)
    got = orc.central_accel(*(np.array([v]) for v in p), G, MC, J2=J2, R_central=RC)[0] - \
        orc.central_accel(*(np.array([v]) for v in p), G, MC)[0]
    assert np.allclose(got, want, rtol=1e-7, atol=1e-12 * np.abs(want).max())


def test_j2_in_the_equatorial_plane(orc):
    """z = 0: an extra inward pull -3/2 G M R^2 J2 / r^4 along r."""
    r = 4.0
    p = np.array([r * math.cos(0.3), r * math.sin(0.3), 0.0])
    got = orc.central_accel(*(np.array([v]) for v in p), G, MC, J2=J2, R_central=RC)[0] - \
        orc.central_accel(*(np.array([v]) for v in p), G, MC)[0]
    want = -1.5 * G * MC * RC * RC * J2 / r ** 4 * p / r
    assert np.allclose(got, want, rtol=1e-9, atol=0)   # got carries the central term's rounding


@pytest.mark.parametrize("t", [0.0, 37.5, 1234.0])
def test_tide_is_minus_gradient_of_its_potential(orc, t):
    s = np.array(orc.sun_position(t, G, MS, AS, EPS))
    assert np.linalg.norm(s) == pytest.approx(AS, rel=1e-14)
    # the orbit stays in the plane tilted by the obliquity about x
    assert s @ np.array([0.0, -math.sin(EPS), math.cos(EPS)]) == pytest.approx(0.0, abs=1e-9)
    p = np.array([5.0, -3.0, 1.0])

    def V(q):                      # -G M_s / (2 a^3) (3 (q.s)^2 / a^2 - q^2)
        return -G * MS / (2 * AS ** 3) * (3 * (q @ s) ** 2 / AS ** 2 - q @ q)

    want = -_num_grad(V, p, 1e-4)
    got = _acc(orc, p, M_sun=MS, a_sun=AS, obliquity=EPS, t=t)
    assert np.allclose(got, want, rtol=1e-7, atol=1e-9 * np.abs(want).max())


def test_tide_approximates_the_differential_attraction(orc):
    """The quadrupolar tide is the exact differential attraction of the distant body
    to first order in r / a: the remainder is O(r / a) relative."""
    t = 10.0
    s = np.array(orc.sun_position(t, G, MS, AS, EPS))
    for p in (np.array([5.0, -3.0, 1.0]), np.array([-8.0, 2.0, -4.0])):
        d = s - p
        exact = G * MS * (d / np.linalg.norm(d) ** 3 - s / AS ** 3)
        got = _acc(orc, p, M_sun=MS, a_sun=AS, obliquity=EPS, t=t)
        ratio = np.linalg.norm(p) / AS
        assert np.linalg.norm(got - exact) <= 3 * ratio * np.linalg.norm(got)
        assert np.linalg.norm(got - exact) >= 1e-3 * ratio * np.linalg.norm(got)

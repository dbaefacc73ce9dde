"""Seeded synthetic workloads for the falcON tree step.

This module only draws inputs; it holds none of the method's arithmetic (no keys,
no tree, no forces, no pair test), so both the CPU oracle and the GPU path can use
it without sharing any of the computation they are compared on.

Workloads (the paper uses synthetic disks only; no public dataset is involved):

* ``disk``      -- moonlets on Keplerian orbits around a central mass of 1 (G = 1,
                   Earth radius 1).  Masses lognormal(0, 1) scaled to a total of
                   0.01; a ~ U[2.9, 10]; e ~ Rayleigh(0.01); i ~ Rayleigh(0.005) rad;
                   Omega, omega, M ~ U[0, 2pi).  Radii from a bulk density of
                   3.3 g/cc expressed in Earth units (Sect. 5: all moonlets share
                   one density).
* ``hot_disk``  -- the disk of the paper's timing runs (Sect. 4.2): a ~ U[2.9, 12],
                   e ~ U[0, 0.2], i ~ U[0, 10 deg].
* ``fig4_disk`` -- the accuracy workload of Fig. 4: a in [1, 10], total mass 0.024.
* ``plummer_sphere`` -- an isolated Plummer sphere of equal masses.
* ``gas_box``   -- a unit box of equal spheres with Maxwellian velocities, used to
                   exercise the collision test (a closed-form pair count exists).
* ``clumps``    -- half a disk plus 200 Plummer spheres placed on disk orbits.
* ``disk_batch`` -- many independent disks (sizes log-uniform, ``batch_sizes``)
                   concatenated, with the offsets of each disk.
"""
from __future__ import annotations

import math

import numpy as np

# Earth mass and radius used to express 3.3 g/cc in units where M_E = R_E = 1.
_EARTH_MASS_G = 5.9722e27
_EARTH_RADIUS_CM = 6.371e8
DENSITY_CODE = 3.3 / (_EARTH_MASS_G / _EARTH_RADIUS_CM ** 3)   # ~0.142890

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "R")


def radius_from_mass(m: np.ndarray, rho: float = DENSITY_CODE) -> np.ndarray:
    return np.cbrt(3.0 * m / (4.0 * math.pi * rho))


def _solve_kepler(M: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Eccentric anomaly E with E - e sin E = M (Newton, to ~1e-15)."""
    E = M + e * np.sin(M)
    for _ in range(50):
        f = E - e * np.sin(E) - M
        dE = f / (1.0 - e * np.cos(E))
        E = E - dE
        if np.max(np.abs(dE)) < 1e-15:
            break
    return E


def elements_to_state(a, e, inc, Om, om, M, mu=1.0):
    """Keplerian elements -> inertial position and velocity (perifocal frame
    rotated by R_z(Omega) R_x(i) R_z(omega))."""
    E = _solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    sq = np.sqrt(1.0 - e * e)
    # perifocal position and velocity
    xp = a * (cE - e)
    yp = a * sq * sE
    r = a * (1.0 - e * cE)
    n = np.sqrt(mu / a ** 3)
    vxp = -a * n * sE * a / r
    vyp = a * n * sq * cE * a / r
    cO, sO = np.cos(Om), np.sin(Om)
    co, so = np.cos(om), np.sin(om)
    ci, si = np.cos(inc), np.sin(inc)
    # rotation matrix R_z(Om) R_x(i) R_z(om), first two columns
    r11 = cO * co - sO * so * ci
    r12 = -cO * so - sO * co * ci
    r21 = sO * co + cO * so * ci
    r22 = -sO * so + cO * co * ci
    r31 = so * si
    r32 = co * si
    pos = (r11 * xp + r12 * yp, r21 * xp + r22 * yp, r31 * xp + r32 * yp)
    vel = (r11 * vxp + r12 * vyp, r21 * vxp + r22 * vyp, r31 * vxp + r32 * vyp)
    return pos, vel


def _pack(pos, vel, m, R):
    out = {
        "x": pos[0], "y": pos[1], "z": pos[2],
        "vx": vel[0], "vy": vel[1], "vz": vel[2],
        "m": m, "R": R,
    }
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in out.items()}


def disk(n: int, seed: int = 0, total_mass: float = 0.01, a_range=(2.9, 10.0),
         e_sigma: float = 0.01, i_sigma: float = 0.005, mu: float = 1.0):
    """The cold disk of moonlets.  Draw order: m, a, e, i, Omega, omega, M."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.lognormal(0.0, 1.0, n)
    m *= total_mass / m.sum()
    a = rng.uniform(a_range[0], a_range[1], n)
    e = rng.rayleigh(e_sigma, n)
    e = np.minimum(e, 0.9)
    inc = rng.rayleigh(i_sigma, n)
    Om = rng.uniform(0.0, 2 * math.pi, n)
    om = rng.uniform(0.0, 2 * math.pi, n)
    M = rng.uniform(0.0, 2 * math.pi, n)
    pos, vel = elements_to_state(a, e, inc, Om, om, M, mu)
    return _pack(pos, vel, m, radius_from_mass(m))


def hot_disk(n: int, seed: int = 0, total_mass: float = 0.01, mu: float = 1.0):
    """The disk of the paper's timing runs: a in [2.9, 12], e in [0, 0.2],
    i in [0, 10 deg], angles uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.lognormal(0.0, 1.0, n)
    m *= total_mass / m.sum()
    a = rng.uniform(2.9, 12.0, n)
    e = rng.uniform(0.0, 0.2, n)
    inc = rng.uniform(0.0, math.radians(10.0), n)
    Om = rng.uniform(0.0, 2 * math.pi, n)
    om = rng.uniform(0.0, 2 * math.pi, n)
    M = rng.uniform(0.0, 2 * math.pi, n)
    pos, vel = elements_to_state(a, e, inc, Om, om, M, mu)
    return _pack(pos, vel, m, radius_from_mass(m))


def fig4_disk(n: int, seed: int = 0, total_mass: float = 0.024, mu: float = 1.0):
    """The accuracy workload of the paper's error distributions (Fig. 4, Sect. 3.4.3):
    moonlets between 1 and 10 Earth radii with random masses totalling 0.024 Earth
    masses.  The paper states neither eccentricities nor inclinations there; this
    reading takes those of its timing runs (e ~ U[0, 0.2], i ~ U[0, 10 deg]) and
    a ~ U[1, 10]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.lognormal(0.0, 1.0, n)
    m *= total_mass / m.sum()
    a = rng.uniform(1.0, 10.0, n)
    e = rng.uniform(0.0, 0.2, n)
    inc = rng.uniform(0.0, math.radians(10.0), n)
    Om = rng.uniform(0.0, 2 * math.pi, n)
    om = rng.uniform(0.0, 2 * math.pi, n)
    M = rng.uniform(0.0, 2 * math.pi, n)
    pos, vel = elements_to_state(a, e, inc, Om, om, M, mu)
    return _pack(pos, vel, m, radius_from_mass(m))


def plummer_sphere(n: int, seed: int = 0, scale: float = 1.0, total_mass: float = 1.0):
    """An isolated Plummer sphere of n equal masses (scale radius `scale`, truncated at
    10 scale radii), sampled as the clumps of ``clumps`` are."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos, vel = _plummer(rng, n, scale, total_mass)
    m = np.full(n, total_mass / n)
    return _pack(pos, vel, m, radius_from_mass(m))


def gas_box(n: int = 2000, seed: int = 0, radius: float = 0.01, sigma: float = 1.0):
    """Uniform unit box [0,1)^3 of equal spheres, velocities N(0, sigma^2) per axis."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.uniform(0.0, 1.0, (3, n))
    vel = rng.normal(0.0, sigma, (3, n))
    m = np.full(n, 1.0 / n)
    R = np.full(n, radius)
    return _pack(pos, vel, m, R)


def gas_box_expected_pairs(n: int, radius: float, sigma: float, dt: float,
                           volume: float = 1.0) -> float:
    """Expected number of pairs that come into contact within dt for a dilute gas
    of equal spheres: N(N-1)/2 * pi S^2 <|dv|> dt / V, S = 2R, <|dv|> = 4 sigma/sqrt(pi)."""
    S = 2.0 * radius
    mean_dv = 4.0 * sigma / math.sqrt(math.pi)
    return 0.5 * n * (n - 1) * math.pi * S * S * mean_dv * dt / volume


def _plummer(rng, n: int, scale: float, mass: float, G: float = 1.0, cut: float = 10.0):
    """Plummer sphere sampled as in Aarseth, Henon & Wielen (1974): radius from
    the cumulative mass, isotropic directions, speed by rejection from
    g(q) = q^2 (1 - q^2)^(7/2) of the escape speed."""
    r = np.empty(n)
    k = 0
    while k < n:
        X = rng.uniform(0.0, 1.0, n - k)
        rr = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr < cut]
        take = min(len(rr), n - k)
        r[k:k + take] = rr[:take]
        k += take

    def iso(rad):
        cth = rng.uniform(-1.0, 1.0, len(rad))
        phi = rng.uniform(0.0, 2 * math.pi, len(rad))
        sth = np.sqrt(1.0 - cth * cth)
        return rad * sth * np.cos(phi), rad * sth * np.sin(phi), rad * cth

    x, y, z = iso(r)
    q = np.empty(n)
    k = 0
    while k < n:
        m = n - k
        q0 = rng.uniform(0.0, 1.0, m)
        g0 = rng.uniform(0.0, 0.1, m)
        ok = g0 < q0 * q0 * (1.0 - q0 * q0) ** 3.5
        acc = q0[ok]
        take = min(len(acc), m)
        q[k:k + take] = acc[:take]
        k += take
    vesc = np.sqrt(2.0) * (1.0 + r * r) ** (-0.25)
    vx, vy, vz = iso(q * vesc)
    # scale from Henon units (G = M = a = 1) to the clump's scale and mass
    vs = math.sqrt(G * mass / scale)
    return (x * scale, y * scale, z * scale), (vx * vs, vy * vs, vz * vs)


def clumps(n: int, seed: int = 0, n_clumps: int = 200, scale: float = 0.05,
           total_mass: float = 0.01, mu: float = 1.0):
    """Clustered stress workload: n/2 moonlets in the cold disk, n/2 in Plummer
    clumps.  Clump weights follow dN/dM ~ M^-2 on [1, 100]; member counts are
    proportional to the weights (remainder on the largest clump).  Each clump
    centre and bulk velocity is a disk orbit; members share one mass scale and
    the global moonlet mass sums to total_mass."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_disk = n // 2
    n_cl = n - n_disk
    base = disk(n_disk, seed=seed + 7919, total_mass=1.0, mu=mu)
    # clump weights: inverse-CDF sample of M^-2 on [1, 100]
    u = rng.uniform(0.0, 1.0, n_clumps)
    w = 1.0 / (1.0 - u * (1.0 - 1.0 / 100.0))
    cnt = np.floor(w / w.sum() * n_cl).astype(np.int64)
    cnt[np.argmax(w)] += n_cl - cnt.sum()
    centres = disk(n_clumps, seed=seed + 104729, total_mass=1.0, mu=mu)
    m_cl = rng.lognormal(0.0, 1.0, n_cl)
    # every mass is rescaled so that the moonlets sum to total_mass; a clump's
    # internal velocities follow from its members' final mass
    fac = total_mass / (base["m"].sum() + m_cl.sum())
    xs, ys, zs, vxs, vys, vzs = [], [], [], [], [], []
    off = 0
    for k in range(n_clumps):
        c = int(cnt[k])
        if c == 0:
            continue
        pos, vel = _plummer(rng, c, scale, mass=m_cl[off:off + c].sum() * fac, G=1.0)
        xs.append(pos[0] + centres["x"][k]); ys.append(pos[1] + centres["y"][k])
        zs.append(pos[2] + centres["z"][k])
        vxs.append(vel[0] + centres["vx"][k]); vys.append(vel[1] + centres["vy"][k])
        vzs.append(vel[2] + centres["vz"][k])
        off += c
    m_all = np.concatenate([base["m"], m_cl]) * fac
    out = {
        "x": np.concatenate([base["x"]] + xs), "y": np.concatenate([base["y"]] + ys),
        "z": np.concatenate([base["z"]] + zs),
        "vx": np.concatenate([base["vx"]] + vxs), "vy": np.concatenate([base["vy"]] + vys),
        "vz": np.concatenate([base["vz"]] + vzs),
        "m": m_all,
    }
    out["R"] = radius_from_mass(m_all)
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in out.items()}


def coincident(n: int, seed: int = 0, copies: int = 3, stack: int = 40):
    """Degenerate positions: a cold disk whose every moonlet appears `copies` times at
    the same place (equal keys, kept in input order by the stable sort), then `stack`
    moonlets on one point, more than a leaf holds, so the tree ends there in a cell
    at the depth cap."""
    base_n = max(1, -(-(n - stack) // copies))
    base = disk(base_n, seed=seed)
    rep = {k: np.repeat(v, copies)[:max(n - stack, 0)] for k, v in base.items()}
    out = {}
    for k, v in rep.items():
        out[k] = np.concatenate([v, np.full(n - len(v), base[k][0])])
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in out.items()}


def batch_sizes(n_disks: int = 64, seed: int = 0, lo: int = 1000, hi: int = 50000):
    """Per-disk sizes, log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_disks))).astype(np.int64)


def disk_batch(sizes, seed_base: int = 1000, kind: str = "disk"):
    """Independent disks concatenated: disk k has sizes[k] moonlets drawn with seed
    seed_base + k (each with its own total mass and central mass at the origin).
    Returns (arrays, offsets) with offsets[k] = first moonlet of disk k and
    offsets[-1] = total.  Empty disks are allowed."""
    gen = {"disk": disk, "hot_disk": hot_disk}[kind]
    parts = []
    for k, nk in enumerate(int(v) for v in sizes):
        if nk > 0:
            parts.append(gen(nk, seed=seed_base + k))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(np.asarray(sizes, dtype=np.int64))
    if parts:
        out = {key: np.concatenate([p_[key] for p_ in parts]) for key in FIELDS}
    else:
        out = {key: np.zeros(0) for key in FIELDS}
    return {k: np.ascontiguousarray(v, dtype=np.float64) for k, v in out.items()}, offsets


def sample_targets(n: int, count: int = 4096, seed: int = 12345) -> np.ndarray:
    """Sorted distinct particle indices used for sampled direct-sum checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    count = min(count, n)
    return np.sort(rng.choice(n, size=count, replace=False)).astype(np.int64)

"""CPU oracle for the falcON tree step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and shares
no code with it.  The arithmetic lives in ``ncorp_oracle.c`` (plain C, FP64);
this file only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ncorp_oracle.c")
_LIB = os.path.join(_HERE, "libncorp_oracle.so")
_lib = None

_f64 = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32 = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u64 = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP for the plain sums)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is not None:
        return _lib
    build()
    L = C.CDLL(_LIB)
    d, i64, i32, vp = C.c_double, C.c_int64, C.c_int, C.c_void_p
    L.orc_pair_test.restype = C.c_int
    L.orc_pair_test.argtypes = [d] * 15
    L.orc_collision_time.restype = d
    L.orc_collision_time.argtypes = [d] * 15
    L.orc_resolve.restype = i64
    L.orc_resolve.argtypes = [i64, _i64, i64, _f64, _f64, _f64, _f64, _f64, _f64, _f64, _f64,
                              d, d, _i32]
    L.orc_mesh_gamma_crit.restype = d
    L.orc_mesh_gamma_crit.argtypes = [d, d, d, d]
    L.orc_mesh_aspect_crit.restype = d
    L.orc_mesh_aspect_crit.argtypes = [d, d]
    L.orc_mesh_gamma_next.restype = d
    L.orc_mesh_gamma_next.argtypes = [d, d, d, d]
    L.orc_mesh_flags.restype = None
    L.orc_mesh_flags.argtypes = [_f64, _f64, i64, d, _i32]
    L.orc_mesh_neighbours.restype = d
    L.orc_mesh_neighbours.argtypes = [_f64, _f64, _f64, _f64, i64, d]
    L.orc_mesh_accel.restype = None
    L.orc_mesh_accel.argtypes = [_f64, _f64, _f64, _f64, _f64, i64, d, d, _f64, _f64, _f64]
    L.orc_mesh_pairs.restype = i64
    L.orc_mesh_pairs.argtypes = [_f64] * 8 + [i64, d, d, _i64, i64]
    L.orc_grav_run_std_targets.restype = None
    L.orc_grav_run_std_targets.argtypes = [vp, i32, i32, _i64, i64, _f64]
    L.orc_mesh_accel_targets.restype = None
    L.orc_mesh_accel_targets.argtypes = [_f64] * 5 + [i64, d, d, _i64, i64, _f64]
    L.orc_mesh_pairs_of.restype = i64
    L.orc_mesh_pairs_of.argtypes = [_f64] * 8 + [i64, d, d, _i64, i64, _i64, i64]
    L.orc_grav_run_std.restype = None
    L.orc_grav_run_std.argtypes = [vp, i32, i32]
    L.orc_root_half_width.restype = d
    L.orc_root_half_width.argtypes = [_f64, _f64, _f64, i64]
    L.orc_quantize.restype = C.c_uint32
    L.orc_quantize.argtypes = [d, d]
    L.orc_hilbert_index.restype = C.c_uint64
    L.orc_hilbert_index.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, i32]
    L.orc_hilbert_keys.restype = None
    L.orc_hilbert_keys.argtypes = [_f64, _f64, _f64, i64, d, _u64]
    L.orc_tree_build.restype = vp
    L.orc_tree_build.argtypes = [_f64, _f64, _f64, i64, d, i32]
    L.orc_tree_free.restype = None
    L.orc_tree_free.argtypes = [vp]
    L.orc_tree_ncells.restype = i64
    L.orc_tree_ncells.argtypes = [vp]
    L.orc_tree_maxlevel.restype = i32
    L.orc_tree_maxlevel.argtypes = [vp]
    L.orc_tree_export.restype = None
    L.orc_tree_export.argtypes = [vp, _i32, _i32, _i32, _i32, _i32, _i32, _u64, _i64, _u64]
    L.orc_theta_of_mass.restype = d
    L.orc_theta_of_mass.argtypes = [d, d, d]
    L.orc_green_derivs.restype = None
    L.orc_green_derivs.argtypes = [_f64, i32, _f64]
    L.orc_green_deriv_full.restype = None
    L.orc_green_deriv_full.argtypes = [_f64, i32, _f64]
    L.orc_grav_new.restype = vp
    L.orc_grav_new.argtypes = [vp, _f64, _f64, _f64, _f64, d, i32, d, i32]
    L.orc_grav_run.restype = None
    L.orc_grav_run.argtypes = [vp, i32, i32, i32]
    L.orc_grav_accel.restype = None
    L.orc_grav_accel.argtypes = [vp, _f64, _f64, _f64]
    L.orc_grav_counts.restype = None
    L.orc_grav_counts.argtypes = [vp, _i64]
    L.orc_grav_lists.restype = None
    L.orc_grav_lists.argtypes = [vp, _i32, _i32]
    L.orc_grav_cells.restype = None
    L.orc_grav_cells.argtypes = [vp, _f64, _f64, _f64, _f64]
    L.orc_grav_msize.restype = i32
    L.orc_grav_msize.argtypes = [vp]
    L.orc_grav_csize.restype = i32
    L.orc_grav_csize.argtypes = [vp]
    L.orc_grav_cell_tensors.restype = None
    L.orc_grav_cell_tensors.argtypes = [vp, i64, _f64, _f64]
    L.orc_grav_free.restype = None
    L.orc_grav_free.argtypes = [vp]
    L.orc_expansion_field.restype = None
    L.orc_expansion_field.argtypes = [_f64, _f64, _f64, _f64, i64, _f64, _f64, _f64, _f64,
                                      i64, i32, _f64, _f64, _f64]
    L.orc_shift_C.restype = None
    L.orc_shift_C.argtypes = [_f64, i32, _f64, _f64]
    L.orc_coll_new.restype = vp
    L.orc_coll_new.argtypes = [vp, _f64, _f64, _f64, _f64, _f64, _f64, _f64, d]
    L.orc_coll_run.restype = i64
    L.orc_coll_run.argtypes = [vp, i32, i32, i32]
    L.orc_coll_pairs.restype = None
    L.orc_coll_pairs.argtypes = [vp, _i64]
    L.orc_coll_ncand.restype = i64
    L.orc_coll_ncand.argtypes = [vp]
    L.orc_coll_ntests.restype = i64
    L.orc_coll_ntests.argtypes = [vp]
    L.orc_coll_cand.restype = None
    L.orc_coll_cand.argtypes = [vp, _i32]
    L.orc_coll_cells.restype = None
    L.orc_coll_cells.argtypes = [vp, _f64, _f64, _f64]
    L.orc_coll_free.restype = None
    L.orc_coll_free.argtypes = [vp]
    L.orc_direct_sum.restype = None
    L.orc_direct_sum.argtypes = [_f64, _f64, _f64, _f64, i64, d, _i64, i64, _f64, _f64, _f64]
    L.orc_pairs_brute.restype = i64
    L.orc_pairs_brute.argtypes = [_f64] * 7 + [i64, d, _i64, i64]
    L.orc_pairs_grid.restype = i64
    L.orc_pairs_grid.argtypes = [_f64] * 7 + [i64, d, _i64, i64]
    L.orc_pairs_of.restype = i64
    L.orc_pairs_of.argtypes = [_f64] * 7 + [i64, d, _i64, i64, _i64, i64]
    _lib = L
    return L


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------- plain pieces
def pair_test(r1, v1, R1, r2, v2, R2, dt) -> bool:
    return bool(lib().orc_pair_test(*map(float, r1), *map(float, v1), float(R1),
                                    *map(float, r2), *map(float, v2), float(R2), float(dt)))


def collision_time(r1, v1, R1, r2, v2, R2, dt) -> float:
    """dt_c of Eq. (2) if the pair collides within [0, dt], else -1."""
    return lib().orc_collision_time(*map(float, r1), *map(float, v1), float(R1),
                                    *map(float, r2), *map(float, v2), float(R2), float(dt))


def resolve(s: dict, pairs, dt: float, f: float = 2.0) -> np.ndarray:
    """Resolves the colliding pairs (rows i < j) of state s in place (Sect. 5.1-5.2,
    greedy in increasing contact time); returns the resolved rows, sorted."""
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    n = len(s["x"])
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        s[k] = np.ascontiguousarray(s[k], dtype=np.float64)
    flags = np.zeros(len(pairs), np.int32)
    lib().orc_resolve(len(pairs), pairs, n, s["x"], s["y"], s["z"], s["vx"], s["vy"], s["vz"],
                      _c(s["m"]), _c(s["R"]), float(dt), float(f), flags)
    return pairs[flags == 1]


def root_half_width(x, y, z) -> float:
    return lib().orc_root_half_width(_c(x), _c(y), _c(z), len(x))


def quantize(v: float, L: float) -> int:
    return int(lib().orc_quantize(float(v), float(L)))


def hilbert_index(cx: int, cy: int, cz: int, bits: int) -> int:
    return int(lib().orc_hilbert_index(cx, cy, cz, bits))


def hilbert_keys(x, y, z, L: float) -> np.ndarray:
    out = np.empty(len(x), dtype=np.uint64)
    lib().orc_hilbert_keys(_c(x), _c(y), _c(z), len(x), float(L), out)
    return out


def theta_of_mass(M: float, M_root: float, theta_min: float) -> float:
    return lib().orc_theta_of_mass(float(M), float(M_root), float(theta_min))


def green_derivs(R, nmax: int) -> np.ndarray:
    """D[a, b, c] = d^a/dx^a d^b/dy^b d^c/dz^c (1/|R|), zero above total order nmax."""
    out = np.zeros(7 ** 3)
    lib().orc_green_derivs(_c(R), nmax, out)
    return out.reshape(7, 7, 7)


def green_deriv_full(R, n: int) -> np.ndarray:
    out = np.zeros(3 ** n)
    lib().orc_green_deriv_full(_c(R), n, out)
    return out.reshape((3,) * n) if n > 0 else out


def expansion_field(src_pos, src_mu, sA, tgt_pos, p: int):
    xs, ys, zs = (_c(src_pos[:, k]) for k in range(3))
    xt, yt, zt = (_c(tgt_pos[:, k]) for k in range(3))
    nt = len(xt)
    ax, ay, az = np.zeros(nt), np.zeros(nt), np.zeros(nt)
    lib().orc_expansion_field(xs, ys, zs, _c(src_mu), len(xs), _c(sA), xt, yt, zt, nt, p,
                              ax, ay, az)
    return np.stack([ax, ay, az], axis=1)


def shift_C(Cin, p: int, d) -> np.ndarray:
    out = np.zeros_like(_c(Cin))
    lib().orc_shift_C(_c(Cin), p, _c(d), out)
    return out


# ---------------------------------------------------------------- tree
class Tree:
    """Pointer-insertion octree, flattened by level then Hilbert order."""

    def __init__(self, x, y, z, s: int, L: float | None = None):
        self.x, self.y, self.z = _c(x), _c(y), _c(z)
        self.n = len(self.x)
        self.L = root_half_width(self.x, self.y, self.z) if L is None else float(L)
        self.s = s
        self._h = lib().orc_tree_build(self.x, self.y, self.z, self.n, self.L, s)
        if not self._h:
            raise ValueError("oracle tree build rejected its arguments")
        nc = lib().orc_tree_ncells(self._h)
        self.ncells = nc
        self.maxlevel = lib().orc_tree_maxlevel(self._h)
        self.level = np.empty(nc, np.int32)
        self.first = np.empty(nc, np.int32)
        self.count = np.empty(nc, np.int32)
        self.child_first = np.empty(nc, np.int32)
        self.nchild = np.empty(nc, np.int32)
        self.parent = np.empty(nc, np.int32)
        self.prefix = np.empty(nc, np.uint64)
        self.perm = np.empty(self.n, np.int64)
        self.keys = np.empty(self.n, np.uint64)
        lib().orc_tree_export(self._h, self.level, self.first, self.count, self.child_first,
                              self.nchild, self.parent, self.prefix, self.perm, self.keys)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc_tree_free(h)
            except Exception:          # interpreter shutdown
                pass
            self._h = None


class Gravity:
    """Climb + TreeWalk + descent of the oracle tree (FP64, full tensors)."""

    def __init__(self, tree: Tree, m, G: float = 1.0, p: int = 3, theta_min: float = 0.5,
                 theta_mode: int = 0):
        self.tree = tree
        self.p = p
        self._h = lib().orc_grav_new(tree._h, tree.x, tree.y, tree.z, _c(m), float(G), p,
                                     float(theta_min), theta_mode)

    def run(self, ncs: int, ncc_pre: int, ncc_post: int):
        lib().orc_grav_run(self._h, ncs, ncc_pre, ncc_post)
        return self

    def run_standard(self, ncb_pre: int, ncb_post: int):
        """The standard tree code (Alg. 1) instead of the falcON walk."""
        lib().orc_grav_run_std(self._h, ncb_pre, ncb_post)
        return self

    def standard_targets(self, ncb_pre: int, ncb_post: int, targets) -> np.ndarray:
        """Standard-tree accelerations of the given moonlets only (input indices)."""
        t = _c(targets, np.int64)
        out = np.zeros((len(t), 3))
        lib().orc_grav_run_std_targets(self._h, ncb_pre, ncb_post, t, len(t), out)
        return out

    def accel(self) -> np.ndarray:
        n = self.tree.n
        ax, ay, az = np.zeros(n), np.zeros(n), np.zeros(n)
        lib().orc_grav_accel(self._h, ax, ay, az)
        return np.stack([ax, ay, az], axis=1)

    def counts(self):
        out = np.zeros(3, np.int64)
        lib().orc_grav_counts(self._h, out)
        return {"m2l": int(out[0]), "p2p": int(out[1]), "p2p_moonlet_pairs": int(out[2])}

    def lists(self):
        c = self.counts()
        m2l = np.zeros((max(c["m2l"], 1), 2), np.int32)
        p2p = np.zeros((max(c["p2p"], 1), 2), np.int32)
        lib().orc_grav_lists(self._h, m2l, p2p)
        return m2l[: c["m2l"]], p2p[: c["p2p"]]

    def cells(self):
        nc = self.tree.ncells
        s = np.zeros((nc, 3)); mass = np.zeros(nc); rmax = np.zeros(nc); rcrit = np.zeros(nc)
        lib().orc_grav_cells(self._h, s, mass, rmax, rcrit)
        return {"s": s, "mass": mass, "rmax": rmax, "rcrit": rcrit}

    def cell_tensors(self, c: int):
        ms, cs = lib().orc_grav_msize(self._h), lib().orc_grav_csize(self._h)
        M = np.zeros(max(ms, 1)); Cc = np.zeros(max(cs, 1))
        lib().orc_grav_cell_tensors(self._h, int(c), M, Cc)
        return M[:ms], Cc[:cs]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc_grav_free(h)
            except Exception:          # interpreter shutdown
                pass
            self._h = None


class Collide:
    """Collision climb + TreeWalk with collision semantics on the oracle tree."""

    def __init__(self, tree: Tree, vx, vy, vz, R, dt: float):
        self.tree = tree
        self._h = lib().orc_coll_new(tree._h, tree.x, tree.y, tree.z, _c(vx), _c(vy), _c(vz),
                                     _c(R), float(dt))

    def run(self, ncs: int = 12, ncc_pre: int = 0, ncc_post: int = 16) -> np.ndarray:
        n = lib().orc_coll_run(self._h, ncs, ncc_pre, ncc_post)
        out = np.zeros((max(n, 1), 2), np.int64)
        lib().orc_coll_pairs(self._h, out)
        return out[:n]

    def candidates(self) -> np.ndarray:
        k = lib().orc_coll_ncand(self._h)
        out = np.zeros((max(k, 1), 2), np.int32)
        lib().orc_coll_cand(self._h, out)
        return out[:k]

    def ntests(self) -> int:
        return int(lib().orc_coll_ntests(self._h))

    def cells(self):
        nc = self.tree.ncells
        sbar = np.zeros((nc, 3)); rmax = np.zeros(nc); rcrit = np.zeros(nc)
        lib().orc_coll_cells(self._h, sbar, rmax, rcrit)
        return {"sbar": sbar, "rmax": rmax, "rcrit": rcrit}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            try:
                _lib.orc_coll_free(h)
            except Exception:          # interpreter shutdown
                pass
            self._h = None


# ---------------------------------------------------------------- plain sums
def direct_sum(x, y, z, m, G: float = 1.0, targets=None) -> np.ndarray:
    n = len(x)
    t = np.arange(n, dtype=np.int64) if targets is None else _c(targets, np.int64)
    ax, ay, az = np.zeros(len(t)), np.zeros(len(t)), np.zeros(len(t))
    lib().orc_direct_sum(_c(x), _c(y), _c(z), _c(m), n, float(G), t, len(t), ax, ay, az)
    return np.stack([ax, ay, az], axis=1)


def pairs_brute(d: dict, dt: float, cap: int = 1 << 20) -> np.ndarray:
    n = len(d["x"])
    out = np.zeros((cap, 2), np.int64)
    k = lib().orc_pairs_brute(*(_c(d[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "R")), n,
                              float(dt), out, cap)
    if k > cap:
        return pairs_brute(d, dt, cap=int(k))
    return out[:k]


def pairs_grid(d: dict, dt: float, cap: int = 1 << 20) -> np.ndarray:
    """Every colliding pair (i < j) of Eqs. (1)-(2), candidates taken from a uniform
    grid of cells wider than twice the largest reach R + dt |v| (the same set as
    pairs_brute, in O(N) for spread-out inputs)."""
    n = len(d["x"])
    out = np.zeros((cap, 2), np.int64)
    k = lib().orc_pairs_grid(*(_c(d[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "R")), n,
                             float(dt), out, cap)
    if k > cap:
        return pairs_grid(d, dt, cap=int(k))
    return out[:k]


def pairs_of(d: dict, dt: float, targets, cap: int = 1 << 20) -> np.ndarray:
    n = len(d["x"])
    t = _c(targets, np.int64)
    out = np.zeros((cap, 2), np.int64)
    k = lib().orc_pairs_of(*(_c(d[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "R")), n,
                           float(dt), t, len(t), out, cap)
    if k > cap:
        return pairs_of(d, dt, targets, cap=int(k))
    res = out[:k]
    if len(res):
        res = np.unique(res, axis=0)
    return res


def sun_position(t: float, G: float, M_sun: float, a_sun: float, obliquity: float):
    """Distant body on a circular orbit of radius a_sun, tilted by the obliquity about
    x, at longitude n t with n = sqrt(G M_sun / a_sun^3) (App. B)."""
    lam = t * math.sqrt(G * M_sun / (a_sun * a_sun * a_sun))
    return (a_sun * math.cos(lam), a_sun * math.sin(lam) * math.cos(obliquity),
            a_sun * math.sin(lam) * math.sin(obliquity))


def central_accel(x, y, z, G: float = 1.0, M_central: float = 1.0, J2: float = 0.0,
                  R_central: float = 1.0, M_sun: float = 0.0, a_sun: float = 0.0,
                  obliquity: float = 0.0, t: float = 0.0) -> np.ndarray:
    """-G M_c r / |r|^3 (App. B.1), plus the central body's J2 bulge
    G M_c R^2 J2 / r^5 [(15 z^2 - 3 r^2) / (2 r^2) r - 3 z e_z] and the quadrupolar
    tide of a distant body -G M_sun / a^3 (r - 3 (r . r_sun) / a^2 r_sun) (App. B)."""
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    f = -(G * M_central) / (r2 * r)
    ax, ay, az = f * x, f * y, f * z
    if J2 != 0.0:
        c = (G * M_central * R_central * R_central * J2) / (r2 * r2 * r)
        k = (15.0 * z * z - 3.0 * r2) / (2.0 * r2)
        ax = ax + c * (k * x)
        ay = ay + c * (k * y)
        az = az + c * (k * z - 3.0 * z)
    if M_sun > 0.0:
        sx, sy, sz = sun_position(t, G, M_sun, a_sun, obliquity)
        q = 3.0 * (x * sx + y * sy + z * sz) / (a_sun * a_sun)
        g = -(G * M_sun) / (a_sun * a_sun * a_sun)
        ax = ax + g * (x - q * sx)
        ay = ay + g * (y - q * sy)
        az = az + g * (z - q * sz)
    return np.stack([ax, ay, az], axis=1)


def tree_accel(d: dict, G=1.0, p=3, theta_min=0.5, s=16, ncs=64, ncc_pre=8, ncc_post=64,
               theta_mode=0, L=None):
    """Mutual accelerations by the oracle falcON tree, input order."""
    t = Tree(d["x"], d["y"], d["z"], s, L)
    g = Gravity(t, d["m"], G, p, theta_min, theta_mode).run(ncs, ncc_pre, ncc_post)
    return g.accel(), t, g


def standard_tree_accel(d: dict, G=1.0, p=3, theta_min=0.5, s=102, ncb_pre=6, ncb_post=16,
                        theta_mode=0, L=None):
    """Mutual accelerations by the oracle's standard tree code (Alg. 1), input order."""
    t = Tree(d["x"], d["y"], d["z"], s, L)
    g = Gravity(t, d["m"], G, p, theta_min, theta_mode).run_standard(ncb_pre, ncb_post)
    return g.accel(), t, g


# ---------------------------------------------------------------- mesh module
def mesh_gamma_crit(x: float, N: float, aspect: float, R_max: float) -> float:
    """Eq. (4): mesh size for x neighbours on average in a disk of aspect h/r."""
    return lib().orc_mesh_gamma_crit(float(x), float(N), float(aspect), float(R_max))


def mesh_aspect_crit(x: float, moon_over_rmax: float) -> float:
    """Eq. (5): smallest h/r for which moonlets of one Moon mass in total fit the mesh."""
    return lib().orc_mesh_aspect_crit(float(x), float(moon_over_rmax))


def mesh_gamma_next(gamma_prev: float, x: float, x_measured: float,
                    gamma_min: float = 0.0) -> float:
    """Eq. (6), clamped below by gamma_min (x' = 0 doubles the mesh)."""
    return lib().orc_mesh_gamma_next(float(gamma_prev), float(x), float(x_measured),
                                     float(gamma_min))


def mesh_flags(m, R, gamma: float) -> np.ndarray:
    """1: out of the mesh (2R > gamma); 2: one of the three most massive; 3: both."""
    n = len(m)
    out = np.zeros(n, np.int32)
    lib().orc_mesh_flags(_c(m), _c(R), n, float(gamma), out)
    return out


def mesh_neighbours(d: dict, gamma: float) -> float:
    """x' of Eq. (6): mean number of other moonlets in a mesh moonlet's neighbourhood."""
    return lib().orc_mesh_neighbours(_c(d["x"]), _c(d["y"]), _c(d["z"]), _c(d["R"]),
                                     len(d["x"]), float(gamma))


def mesh_accel(d: dict, gamma: float, G: float = 1.0) -> np.ndarray:
    """Mutual accelerations of the mesh module (Sect. 3.3), input order."""
    n = len(d["x"])
    ax, ay, az = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_mesh_accel(_c(d["x"]), _c(d["y"]), _c(d["z"]), _c(d["m"]), _c(d["R"]), n,
                         float(G), float(gamma), ax, ay, az)
    return np.stack([ax, ay, az], axis=1)


def mesh_accel_of(d: dict, gamma: float, targets, G: float = 1.0) -> np.ndarray:
    """Mesh-module accelerations of the given moonlets only (input indices)."""
    t = _c(targets, np.int64)
    out = np.zeros((len(t), 3))
    lib().orc_mesh_accel_targets(_c(d["x"]), _c(d["y"]), _c(d["z"]), _c(d["m"]), _c(d["R"]),
                                 len(d["x"]), float(G), float(gamma), t, len(t), out)
    return out


def mesh_pairs_of(d: dict, gamma: float, dt: float, targets, cap: int = 1 << 20) -> np.ndarray:
    """Colliding mesh pairs that involve one of the targets (sorted, distinct)."""
    t = np.unique(_c(targets, np.int64))
    out = np.zeros((cap, 2), np.int64)
    k = lib().orc_mesh_pairs_of(*(_c(d[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "m", "R")),
                                len(d["x"]), float(gamma), float(dt), t, len(t), out, cap)
    if k > cap:
        return mesh_pairs_of(d, gamma, dt, targets, cap=int(k))
    return out[:k]


def mesh_pairs(d: dict, gamma: float, dt: float, cap: int = 1 << 20) -> np.ndarray:
    """Colliding pairs (i < j, increasing) among the pairs the mesh tests."""
    n = len(d["x"])
    out = np.zeros((cap, 2), np.int64)
    k = lib().orc_mesh_pairs(*(_c(d[f]) for f in ("x", "y", "z", "vx", "vy", "vz", "m", "R")),
                             n, float(gamma), float(dt), out, cap)
    if k > cap:
        return mesh_pairs(d, gamma, dt, cap=int(k))
    return out[:k]


class MeshClock:
    """The mesh size along a run (Sect. 3.3): gamma_0 from Eq. (4) at the first mesh
    (R_max = the largest distance to the central mass unless given), then Eq. (6) from
    the previous mesh's neighbour count at every new mesh.  ``accel`` and ``collide``
    fit ``kdk_steps``: each ``accel`` call builds a new mesh at the current positions,
    and ``collide`` uses the mesh of the last ``accel`` call."""

    def __init__(self, x_target: float, aspect: float, R_max: float = 0.0,
                 gamma_min: float = 0.0, G: float = 1.0, gamma0: float = 0.0):
        self.x, self.aspect, self.R_max, self.gamma_min, self.G = (
            x_target, aspect, R_max, gamma_min, G)
        self.gamma0 = gamma0
        self.gamma = None
        self.measured = None
        self.history = []

    def _new_mesh(self, s):
        if self.gamma is None:
            if self.gamma0 > 0.0:
                g = self.gamma0
            else:
                rmax = self.R_max if self.R_max > 0.0 else float(
                    np.sqrt(s["x"] ** 2 + s["y"] ** 2 + s["z"] ** 2).max())
                g = mesh_gamma_crit(self.x, len(s["x"]), self.aspect, rmax)
            self.gamma = max(g, self.gamma_min)
        else:
            self.gamma = mesh_gamma_next(self.gamma, self.x, self.measured, self.gamma_min)
        self.measured = mesh_neighbours(s, self.gamma)
        self.history.append((self.gamma, self.measured))

    def accel(self, s):
        self._new_mesh(s)
        return mesh_accel(s, self.gamma, self.G)

    def collide(self, s, dt):
        return mesh_pairs(s, self.gamma, dt)


def kdk_steps(d: dict, dt: float, n_steps: int, accel_fn, G=1.0, M_central=1.0,
              collide_fn=None, resolve_f=None, central=None, t_start: float = 0.0):
    """Merged kick-drift-kick leapfrog around the central mass (Sect. 4.1, SBAB1
    form): v += dt/2 a; [collision search on (x, v)]; x += dt v; a = a(x); v += dt/2 a.
    With resolve_f, the pairs found are resolved (``resolve``, coefficient f) before
    the drift and the per-step lists hold the resolved pairs.  ``central`` holds the
    extra keyword arguments of ``central_accel`` (J2, R_central, M_sun, a_sun,
    obliquity); the kicks happen at t_start + k dt.
    Returns the new state and the per-step pair lists."""
    s = {k: np.array(v, dtype=np.float64) for k, v in d.items()}

    extra = dict(central or {})

    def total_acc(t):
        a = central_accel(s["x"], s["y"], s["z"], G, M_central, t=t, **extra)
        if accel_fn is not None:
            a = accel_fn(s) + a
        return a

    a = total_acc(t_start)
    pairs = []
    for k in range(n_steps):
        for c, f in enumerate(("vx", "vy", "vz")):
            s[f] = s[f] + 0.5 * dt * a[:, c]
        if collide_fn is not None:
            found = collide_fn(s, dt)
            if resolve_f is not None:
                found = resolve(s, found, dt, resolve_f)
            pairs.append(found)
        for c, f in enumerate(("x", "y", "z")):
            s[f] = s[f] + dt * s[("vx", "vy", "vz")[c]]
        a = total_acc(t_start + (k + 1) * dt)
        for c, f in enumerate(("vx", "vy", "vz")):
            s[f] = s[f] + 0.5 * dt * a[:, c]
    return s, pairs

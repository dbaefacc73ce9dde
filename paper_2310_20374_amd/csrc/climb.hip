// Tree climbs (Sect. 3.4.2).  One thread per leaf computes the leaf, then walks up:
// each finished cell bumps its parent's arrival counter and the thread that
// arrives last computes the parent from its (complete) children.  No thread ever
// waits, so the pass is a single launch with no level loop.
//
// Gravity: centre of mass (Eq. 10), r_max (Eq. 11) clamped to the farthest corner
// of the cell's cube, scaled multipole moments Mt_a = M_a / a! (Eq. 20 at leaves,
// binomial shift of App. C above), then theta(M) and r_crit = r_max/theta (Eq. 12)
// once the root mass is known.  Collisions: centroid (Eq. 7), r_max (Eq. 8) and
// r_crit (Eq. 9) with r_crit - r_max = R + dt |v| for a moonlet.
//
// Operation order of the centres, radii and angles is fixed (children or moonlets
// in tree order, no contraction) so they are reproducible bit for bit.
#include "ncorp_internal.h"

namespace ncorp {

__device__ __forceinline__ double dist3(double ax, double ay, double az, double bx, double by,
                                        double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ uint32_t quantize_c(double x, double L, double scale) {
    double t = (x + L) * scale;
    if (!(t >= 0.0)) return 0u;
    if (t >= 2097152.0) return 2097151u;
    uint32_t q = (uint32_t)floor(t);
    return q > 2097151u ? 2097151u : q;
}

// distance from (sx, sy, sz) to the farthest corner of the cell's cube; the cube
// follows from any moonlet of the cell (here its first) and the cell's level
__device__ double far_corner(double sx, double sy, double sz, double px, double py, double pz,
                             int level, double L) {
    double scale = 1048576.0 / L;
    int sh = kMaxDepth - level;
    double cx = (double)(quantize_c(px, L, scale) >> sh);
    double cy = (double)(quantize_c(py, L, scale) >> sh);
    double cz = (double)(quantize_c(pz, L, scale) >> sh);
    double hw = ldexp(L, -level);
    double side = ldexp(1.0, level);
    double ex = hw * (2.0 * cx + 1.0 - side);
    double ey = hw * (2.0 * cy + 1.0 - side);
    double ez = hw * (2.0 * cz + 1.0 - side);
    double dx = fabs(sx - ex) + hw, dy = fabs(sy - ey) + hw, dz = fabs(sz - ez) + hw;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ double ld_coherent(const double *p) {
    return __builtin_nontemporal_load(p);
}

template <int P>
struct Mult {
    static constexpr int NM = n_mult(P);
};

// scaled powers u^a / a! for a = 0..P-1 per axis
template <int P>
__device__ __forceinline__ void scaled_powers(double ux, double uy, double uz, double *px,
                                              double *py, double *pz) {
    px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
    for (int a = 1; a < (P > 1 ? P : 1); a++) {
        double inv = 1.0 / (double)a;
        px[a] = px[a - 1] * ux * inv;
        py[a] = py[a - 1] * uy * inv;
        pz[a] = pz[a - 1] * uz * inv;
    }
}

// leaf: moments straight from the moonlets (Eq. 20), scaled by 1/a!
template <int P>
__device__ void leaf_moments(const double *__restrict__ xs, const double *__restrict__ ys,
                             const double *__restrict__ zs, const double *__restrict__ mus,
                             int f, int cnt, double sx, double sy, double sz, double *out) {
    constexpr int NM = n_mult(P);
    double acc[NM > 0 ? NM : 1];
#pragma unroll
    for (int k = 0; k < NM; k++) acc[k] = 0.0;
    for (int k = f; k < f + cnt; k++) {
        double mu = mus[k];
        double px[P > 1 ? P : 1], py[P > 1 ? P : 1], pz[P > 1 ? P : 1];
        scaled_powers<P>(xs[k] - sx, ys[k] - sy, zs[k] - sz, px, py, pz);
#pragma unroll
        for (int n = 0; n < P; n++) {
            if (n == 1) continue;
#pragma unroll
            for (int b = 0; b <= n; b++)
#pragma unroll
                for (int c = 0; c <= n - b; c++) {
                    int a = n - b - c;
                    acc[midx(a, b, c)] += mu * px[a] * py[b] * pz[c];
                }
        }
    }
#pragma unroll
    for (int k = 0; k < NM; k++) out[k] = acc[k];
}

// parent moments: sum over children of the shifted child moments (App. C):
// Mt_a(s_B) = sum_{b <= a} Mt_b(s_b) u^(a-b)/(a-b)!,  u = s_b - s_B
template <int P>
__device__ void shift_add(const double *__restrict__ child, double ux, double uy, double uz,
                          double *acc) {
    double px[P > 1 ? P : 1], py[P > 1 ? P : 1], pz[P > 1 ? P : 1];
    scaled_powers<P>(ux, uy, uz, px, py, pz);
    double m[n_mult(P) > 0 ? n_mult(P) : 1];
#pragma unroll
    for (int k = 0; k < n_mult(P); k++) m[k] = ld_coherent(child + k);
#pragma unroll
    for (int n = 0; n < P; n++) {
        if (n == 1) continue;
#pragma unroll
        for (int b = 0; b <= n; b++)
#pragma unroll
            for (int c = 0; c <= n - b; c++) {
                const int a = n - b - c;
                double s = 0.0;
#pragma unroll
                for (int a2 = 0; a2 <= a; a2++)
#pragma unroll
                    for (int b2 = 0; b2 <= b; b2++)
#pragma unroll
                        for (int c2 = 0; c2 <= c; c2++) {
                            const int n2 = a2 + b2 + c2;
                            if (n2 == 1) continue;
                            s += m[midx(a2, b2, c2)] * (px[a - a2] * py[b - b2] * pz[c - c2]);
                        }
                acc[midx(a, b, c)] += s;
            }
    }
}

template <int P>
__global__ void __launch_bounds__(128)
k_gravity_climb(const DevState *__restrict__ st, const double *__restrict__ xs,
                const double *__restrict__ ys, const double *__restrict__ zs,
                const double *__restrict__ mus, const int32_t *__restrict__ ent_cell,
                const int32_t *__restrict__ c_level, const int32_t *__restrict__ c_first,
                const int32_t *__restrict__ c_count, const int32_t *__restrict__ c_child,
                const int32_t *__restrict__ c_nchild, const int32_t *__restrict__ c_parent,
                int32_t *c_arrive, double4 *gcell, double *c_mass, double *c_rmax,
                double *mult, float *mult32) {
    constexpr int NM = n_mult(P);
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    const double L = st->L;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
        int c = ent_cell[e];
        // ---- leaf
        {
            int f = c_first[c], cnt = c_count[c];
            double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int k = f; k < f + cnt; k++) {
                double mu = mus[k];
                M += mu;
                sx += mu * xs[k];
                sy += mu * ys[k];
                sz += mu * zs[k];
            }
            sx = sx / M; sy = sy / M; sz = sz / M;
            double rm = 0.0;
            for (int k = f; k < f + cnt; k++) {
                double d = 0.0 + dist3(xs[k], ys[k], zs[k], sx, sy, sz);
                if (d > rm) rm = d;
            }
            double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c], L);
            if (fc < rm) rm = fc;
            gcell[c] = make_double4(sx, sy, sz, 0.0);
            c_mass[c] = M;
            c_rmax[c] = rm;
            if (NM > 0) {
                double mt[NM > 0 ? NM : 1];
                leaf_moments<P>(xs, ys, zs, mus, f, cnt, sx, sy, sz, mt);
                double *o = mult + (int64_t)c * NM;
                float *o32 = mult32 + (int64_t)c * NM;
#pragma unroll
                for (int k = 0; k < NM; k++) { o[k] = mt[k]; o32[k] = (float)mt[k]; }
            }
        }
        // ---- walk up while this thread is the last child to arrive
        for (int up = 0; up < kMaxDepth; up++) {      // at most one step per level
            int par = c_parent[c];
            if (par < 0) break;
            __threadfence();
            int old = atomicAdd(&c_arrive[par], 1);
            if (old != c_nchild[par] - 1) break;
            __threadfence();
            c = par;
            int a0 = c_child[c], a1 = a0 + c_nchild[c];
            double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int a = a0; a < a1; a++) M += ld_coherent(&c_mass[a]);
            for (int a = a0; a < a1; a++) {
                double ma = ld_coherent(&c_mass[a]);
                sx += ma * ld_coherent(&gcell[a].x);
                sy += ma * ld_coherent(&gcell[a].y);
                sz += ma * ld_coherent(&gcell[a].z);
            }
            sx = sx / M; sy = sy / M; sz = sz / M;
            double rm = 0.0;
            for (int a = a0; a < a1; a++) {
                double d = ld_coherent(&c_rmax[a]) +
                           dist3(ld_coherent(&gcell[a].x), ld_coherent(&gcell[a].y),
                                 ld_coherent(&gcell[a].z), sx, sy, sz);
                if (d > rm) rm = d;
            }
            int f = c_first[c];
            double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c], L);
            if (fc < rm) rm = fc;
            gcell[c] = make_double4(sx, sy, sz, 0.0);
            c_mass[c] = M;
            c_rmax[c] = rm;
            if (NM > 0) {
                double acc[NM > 0 ? NM : 1];
#pragma unroll
                for (int k = 0; k < NM; k++) acc[k] = 0.0;
                for (int a = a0; a < a1; a++) {
                    double ux = ld_coherent(&gcell[a].x) - sx;
                    double uy = ld_coherent(&gcell[a].y) - sy;
                    double uz = ld_coherent(&gcell[a].z) - sz;
                    shift_add<P>(mult + (int64_t)a * NM, ux, uy, uz, acc);
                }
                double *o = mult + (int64_t)c * NM;
                float *o32 = mult32 + (int64_t)c * NM;
#pragma unroll
                for (int k = 0; k < NM; k++) { o[k] = acc[k]; o32[k] = (float)acc[k]; }
            }
        }
    }
}

// theta(M) of Dehnen's relation, solved with only + - * / (reading R3):
//   theta^15 M = K^3 M_root (1 - theta)^6,  K = theta_min^5 / (1 - theta_min)^2
__device__ double theta_of_mass(double M, double Mroot, double tmin) {
    if (!(M < Mroot)) return tmin;
    double tm = tmin, um = 1.0 - tmin;
    double tm2 = tm * tm, tm4 = tm2 * tm2, tm5 = tm4 * tm;
    double um2 = um * um;
    double K = tm5 / um2;
    double K3 = K * K * K;
    double rhs0 = K3 * Mroot;
    double lo = tmin, hi = 1.0;
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (lo + hi);
        double t2 = mid * mid, t4 = t2 * t2, t8 = t4 * t4;
        double t15 = t8 * t4 * t2 * mid;
        double u = 1.0 - mid, u2 = u * u, u4 = u2 * u2, u6 = u4 * u2;
        double g = t15 * M - rhs0 * u6;
        if (g <= 0.0) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ void k_rcrit(const DevState *__restrict__ st, const double *__restrict__ c_mass,
                        const double *__restrict__ c_rmax, double4 *gcell, double *c_theta,
                        double theta_min, int theta_mode, const int32_t *__restrict__ c_count,
                        const int32_t *__restrict__ c_child, const int32_t *__restrict__ c_nchild,
                        WCell *__restrict__ wg) {
    const int nc = st->ncells;
    if (nc <= 0 || (st->status & kSkipMask)) return;
    const double Mroot = c_mass[0];
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        double th = theta_mode == 1 ? theta_min : theta_of_mass(c_mass[c], Mroot, theta_min);
        c_theta[c] = th;
        const double rc = c_rmax[c] / th;
        double4 g = gcell[c];
        g.w = rc;
        gcell[c] = g;
        WCell w;
        w.x = g.x; w.y = g.y; w.z = g.z; w.rcrit = rc;
        w.count = c_count[c]; w.child = c_child[c]; w.nchild = c_nchild[c]; w.pad = 0;
        wg[c] = w;
    }
}

__global__ void k_pack_collision(const DevState *__restrict__ st, const double4 *__restrict__ ccell,
                                 const int32_t *__restrict__ c_count,
                                 const int32_t *__restrict__ c_child,
                                 const int32_t *__restrict__ c_nchild, WCell *__restrict__ wc) {
    const int nc = st->ncells;
    if (st->status & kSkipMask) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        const double4 g = ccell[c];
        WCell w;
        w.x = g.x; w.y = g.y; w.z = g.z; w.rcrit = g.w;
        w.count = c_count[c]; w.child = c_child[c]; w.nchild = c_nchild[c]; w.pad = 0;
        wc[c] = w;
    }
}

__global__ void k_arrive_reset(const DevState *__restrict__ st, int32_t *c_arrive) {
    const int nc = st->ncells;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
        c_arrive[c] = 0;
}

static int cell_grid(int64_t cap, int block) {
    int64_t g = (cap + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

template <int P>
static void launch_gc(const Workspace &ws, hipStream_t s) {
    int g = cell_grid(ws.n_max, 128);
    k_gravity_climb<P><<<g, 128, 0, s>>>(ws.st, ws.xs, ws.ys, ws.zs, ws.mus, ws.ent_cell,
                                         ws.c_level, ws.c_first, ws.c_count, ws.c_child,
                                         ws.c_nchild, ws.c_parent, ws.c_arrive, ws.gcell,
                                         ws.c_mass, ws.c_rmax, ws.mult, ws.mult32);
}

hipError_t launch_gravity_climb(const Workspace &ws, int64_t n, const ncorp_params &prm,
                                hipStream_t s) {
    (void)n;
    k_arrive_reset<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.c_arrive);
    switch (prm.p) {
        case 0: launch_gc<0>(ws, s); break;
        case 1: launch_gc<1>(ws, s); break;
        case 2: launch_gc<2>(ws, s); break;
        case 3: launch_gc<3>(ws, s); break;
        case 4: launch_gc<4>(ws, s); break;
        case 5: launch_gc<5>(ws, s); break;
        default: launch_gc<6>(ws, s); break;
    }
    k_rcrit<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.c_mass, ws.c_rmax, ws.gcell,
                                                        ws.c_theta, prm.theta_min, prm.theta_mode,
                                                        ws.c_count, ws.c_child, ws.c_nchild, ws.wg);
    return hipGetLastError();
}

// ------------------------------------------------------------------ collisions
__global__ void __launch_bounds__(128)
k_collision_climb(const DevState *__restrict__ st, const double *__restrict__ xs,
                  const double *__restrict__ ys, const double *__restrict__ zs,
                  const double *__restrict__ vxs, const double *__restrict__ vys,
                  const double *__restrict__ vzs, const double *__restrict__ rads, double dt,
                  const int32_t *__restrict__ ent_cell, const int32_t *__restrict__ c_level,
                  const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
                  const int32_t *__restrict__ c_child, const int32_t *__restrict__ c_nchild,
                  const int32_t *__restrict__ c_parent, int32_t *c_arrive, double4 *ccell,
                  double *c_crmax) {
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    const double L = st->L;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
        int c = ent_cell[e];
        {
            int f = c_first[c], cnt = c_count[c];
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int k = f; k < f + cnt; k++) { sx += xs[k]; sy += ys[k]; sz += zs[k]; }
            double NA = (double)cnt;
            sx = sx / NA; sy = sy / NA; sz = sz / NA;
            double rm = 0.0, ex = 0.0;
            for (int k = f; k < f + cnt; k++) {
                double d = 0.0 + dist3(xs[k], ys[k], zs[k], sx, sy, sz);
                if (d > rm) rm = d;
                double v = sqrt(vxs[k] * vxs[k] + vys[k] * vys[k] + vzs[k] * vzs[k]);
                double ee = (rads[k] + dt * v) - 0.0;
                if (ee > ex) ex = ee;
            }
            double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c], L);
            if (fc < rm) rm = fc;
            ccell[c] = make_double4(sx, sy, sz, rm + ex);
            c_crmax[c] = rm;
        }
        for (int up = 0; up < kMaxDepth; up++) {      // at most one step per level
            int par = c_parent[c];
            if (par < 0) break;
            __threadfence();
            int old = atomicAdd(&c_arrive[par], 1);
            if (old != c_nchild[par] - 1) break;
            __threadfence();
            c = par;
            int a0 = c_child[c], a1 = a0 + c_nchild[c];
            double NA = (double)c_count[c];
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int a = a0; a < a1; a++) {
                double na = (double)c_count[a];
                sx += na * ld_coherent(&ccell[a].x);
                sy += na * ld_coherent(&ccell[a].y);
                sz += na * ld_coherent(&ccell[a].z);
            }
            sx = sx / NA; sy = sy / NA; sz = sz / NA;
            double rm = 0.0, ex = 0.0;
            for (int a = a0; a < a1; a++) {
                double rma = ld_coherent(&c_crmax[a]);
                double d = rma + dist3(ld_coherent(&ccell[a].x), ld_coherent(&ccell[a].y),
                                       ld_coherent(&ccell[a].z), sx, sy, sz);
                if (d > rm) rm = d;
                double ee = ld_coherent(&ccell[a].w) - rma;
                if (ee > ex) ex = ee;
            }
            int f = c_first[c];
            double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c], L);
            if (fc < rm) rm = fc;
            ccell[c] = make_double4(sx, sy, sz, rm + ex);
            c_crmax[c] = rm;
        }
    }
}

hipError_t launch_collision_climb(const Workspace &ws, int64_t n, double dt, hipStream_t s) {
    (void)n;
    k_arrive_reset<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.c_arrive);
    k_collision_climb<<<cell_grid(ws.n_max, 128), 128, 0, s>>>(
        ws.st, ws.xs, ws.ys, ws.zs, ws.vxs, ws.vys, ws.vzs, ws.rads, dt, ws.ent_cell, ws.c_level,
        ws.c_first, ws.c_count, ws.c_child, ws.c_nchild, ws.c_parent, ws.c_arrive, ws.ccell,
        ws.c_crmax);
    k_pack_collision<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.ccell, ws.c_count,
                                                                 ws.c_child, ws.c_nchild, ws.wc);
    return hipGetLastError();
}

}  // namespace ncorp

// Mesh module (Sect. 3.3): mutual gravity and collision search restricted to
// moonlets in each other's neighbourhood on a mesh of cubic cells of side gamma,
// plus the moonlets that interact with everyone (too large for the mesh, and for
// gravity the three most massive).
//
// Build: every moonlet gets its cell c = floor(r / gamma) and the hash bucket of
// c in an M^3 table (each coordinate taken modulo M); the moonlets are sorted by
// bucket with a stable radix sort (input order inside a bucket; moonlets kept out
// of the mesh get the key M^3 and end up last), and each bucket records the range
// [first, end) of its moonlets together with the build's stamp, so the table never
// needs clearing.  A neighbourhood scan reads the 27 buckets around a cell and
// keeps the moonlets whose cell is exactly the neighbouring cell (with M >= 3 the
// 27 cells fall into distinct buckets, so a cell that shares a bucket is never a
// neighbour).  Moonlets sorted by bucket sit next to the moonlets of their own
// cell, so the lanes of a wave read overlapping buckets.
//
// The mesh size: Eq. (4) at the first mesh (or the value given), then Eq. (6) from
// the neighbour count of the previous mesh, kept on the device so that a step
// loop (and a captured graph of it) needs no host round trip.
#include "contact.h"

namespace ncorp {
namespace {

constexpr int kMeshBlock = 256;
constexpr int kMeshTopBlocks = 256;
constexpr int kMeshChunks = 64;      // source chunks of the all-pairs sums
constexpr int kMeshBigRows = 16;     // big moonlets handled side by side

__device__ __forceinline__ int64_t wrap(int64_t a, int64_t M) {
    const int64_t r = a % M;
    return r < 0 ? r + M : r;
}

__device__ __forceinline__ int64_t bucket_of(int cx, int cy, int cz, int M) {
    return wrap(cx, M) + (int64_t)M * (wrap(cy, M) + (int64_t)M * wrap(cz, M));
}

// cell of a position; false if a coordinate leaves +-kMeshCellLimit
__device__ __forceinline__ bool cell_of(double x, double y, double z, double g, int4 &c) {
    const double fx = floor(x / g), fy = floor(y / g), fz = floor(z / g);
    const double lim = (double)kMeshCellLimit;
    if (!(fabs(fx) < lim && fabs(fy) < lim && fabs(fz) < lim)) return false;
    c.x = (int)fx; c.y = (int)fy; c.z = (int)fz; c.w = 0;
    return true;
}

__device__ __forceinline__ void add_pull(double4 src, double x, double y, double z, double &a0,
                                         double &a1, double &a2) {
    const double dx = src.x - x, dy = src.y - y, dz = src.z - z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;
    const double r = sqrt(r2), r3 = r2 * r;
    a0 += src.w * dx / r3;
    a1 += src.w * dy / r3;
    a2 += src.w * dz / r3;
}

// ------------------------------------------------------------------ build
__global__ void k_mesh_clear(int4 *tab, int64_t nb, MeshState *ms) {
    for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < nb;
         b += (int64_t)gridDim.x * blockDim.x)
        tab[b] = make_int4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MeshState z = {};
        *ms = z;
    }
}

__global__ void k_mesh_rmax(const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, int64_t n, MeshState *ms) {
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r2 = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
        m = r2 > m ? r2 : m;       // NaN positions are reported by the keys kernel
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    // non-negative doubles order like their bit patterns
    if ((threadIdx.x & (kWave - 1)) == 0)
        atomicMax((unsigned long long *)&ms->rmax2, (unsigned long long)__double_as_longlong(m));
}

// the mesh size of the new mesh (Eq. 4 at the first mesh, Eq. 6 after), new stamp
__global__ void k_mesh_begin(MeshState *ms, DevState *st, int64_t n, double x_target,
                             double aspect, double rmax, double gamma0, double gamma_min) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double g;
    if (!ms->init) {
        if (gamma0 > 0.0) {
            g = gamma0;
        } else {
            const double R = rmax > 0.0 ? rmax : sqrt(ms->rmax2);
            const double s = aspect * aspect / (1.0 + aspect * aspect);
            g = pow(4.0 * 3.14159265358979323846 * x_target / (81.0 * (double)n), 1.0 / 3.0) *
                pow(s, 1.0 / 6.0) * R;
        }
        ms->init = 1;
    } else if (ms->measured) {
        const double xm = ms->n_in > 0 ? (double)ms->nbr_sum / (double)ms->n_in : 0.0;
        g = xm > 0.0 ? ms->gamma * cbrt(x_target / xm) : 2.0 * ms->gamma;
    } else {
        g = ms->gamma;
    }
    if (g < gamma_min) g = gamma_min;
    if (!(g > 0.0) || !(g < INFINITY)) atomicOr(&st->status, (int32_t)ST_MESH_RANGE);
    ms->gamma = g;
    ms->stamp += 1;
    ms->measured = 0;
    ms->nbr_sum = 0;
    ms->n_in = (int32_t)n;
    ms->ntop = 0;
    ms->nbig = 0;
}

__global__ void k_mesh_keys(DevState *st, const MeshState *__restrict__ ms,
                            const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, const double *__restrict__ R, int64_t n,
                            int M, uint64_t *keys, uint32_t *vals) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double g = ms->gamma;
    uint64_t key = (uint64_t)M * M * M;            // out of the mesh: sorted last
    if (!(2.0 * R[i] > g)) {
        int4 c;
        if (cell_of(x[i], y[i], z[i], g, c))
            key = (uint64_t)bucket_of(c.x, c.y, c.z, M);
        else if (isfinite(x[i]) && isfinite(y[i]) && isfinite(z[i]))
            atomicOr(&st->status, (int32_t)ST_MESH_RANGE);
        else
            atomicOr(&st->status, (int32_t)ST_NONFINITE);   // kept out: never indexed
    }
    keys[i] = key;
    vals[i] = (uint32_t)i;
}

// sorted positions, cells, bucket ranges; the first out-of-mesh position is n_in
__global__ void k_mesh_table(DevState *st, MeshState *ms, const uint64_t *__restrict__ keys,
                             const uint32_t *__restrict__ idx, const double *__restrict__ x,
                             const double *__restrict__ y, const double *__restrict__ z,
                             int64_t n, int M, int4 *tab, double4 *mpos, int4 *mcell) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n || (st->status & kSkipMask)) return;
    const uint32_t i = idx[q];
    const double g = ms->gamma;
    mpos[q] = make_double4(x[i], y[i], z[i], 0.0);
    const uint64_t out = (uint64_t)M * M * M;
    const uint64_t k = keys[q];
    if (k == out) {
        if (q == 0 || keys[q - 1] != out) ms->n_in = (int32_t)q;
        mcell[q] = make_int4(0, 0, 0, 0);
        return;
    }
    int4 c;
    cell_of(x[i], y[i], z[i], g, c);               // in range: checked by k_mesh_keys
    mcell[q] = c;
    const int stamp = ms->stamp;
    if (q == 0 || keys[q - 1] != k) {
        tab[k].x = (int)q;
        tab[k].z = stamp;
    }
    if (q == n - 1 || keys[q + 1] != k) tab[k].y = (int)(q + 1);
}

// ------------------------------------------------------------------ gravity
// mu = G m in sorted order
__global__ void k_mesh_mu(const uint32_t *__restrict__ idx, const double *__restrict__ m,
                          double G, int64_t n, double4 *mpos) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) mpos[q].w = G * m[idx[q]];
}

// a before b: larger mass, then smaller input index
__device__ __forceinline__ bool heavier(const double *m, const uint32_t *idx, int a, int b) {
    if (b < 0) return a >= 0;
    if (a < 0) return false;
    const double ma = m[idx[a]], mb = m[idx[b]];
    return ma > mb || (ma == mb && idx[a] < idx[b]);
}

__device__ __forceinline__ void keep_top3(const double *m, const uint32_t *idx, int t[3], int c) {
    if (heavier(m, idx, c, t[0])) { t[2] = t[1]; t[1] = t[0]; t[0] = c; }
    else if (heavier(m, idx, c, t[1])) { t[2] = t[1]; t[1] = c; }
    else if (heavier(m, idx, c, t[2])) t[2] = c;
}

__global__ void __launch_bounds__(kMeshBlock)
k_mesh_top_part(const DevState *__restrict__ st, const double *__restrict__ m,
                const uint32_t *__restrict__ idx, int64_t n, int32_t *part) {
    __shared__ int cand[kMeshBlock * 3];
    if (st->status & kSkipMask) return;
    int t[3] = {-1, -1, -1};
    for (int64_t q = blockIdx.x * (int64_t)kMeshBlock + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kMeshBlock)
        keep_top3(m, idx, t, (int)q);
    for (int k = 0; k < 3; k++) cand[3 * threadIdx.x + k] = t[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        int b[3] = {-1, -1, -1};
        for (int k = 0; k < kMeshBlock * 3; k++) keep_top3(m, idx, b, cand[k]);
        for (int k = 0; k < 3; k++) part[3 * blockIdx.x + k] = b[k];
    }
}

// the three most massive, and gravity's all-pairs list: the moonlets out of the
// mesh (sorted positions n_in..n-1), then the three most massive that are in it
__global__ void k_mesh_top_final(DevState *st, MeshState *ms, const double *__restrict__ m,
                                 const uint32_t *__restrict__ idx, int64_t n,
                                 const int32_t *__restrict__ part, int32_t *big) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || (st->status & kSkipMask)) return;
    int b[3] = {-1, -1, -1};
    for (int k = 0; k < kMeshTopBlocks * 3; k++) keep_top3(m, idx, b, part[k]);
    int ntop = 0;
    for (int k = 0; k < 3; k++)
        if (b[k] >= 0) ms->top[ntop++] = b[k];
    for (int k = ntop; k < 3; k++) ms->top[k] = -1;
    ms->ntop = ntop;
    const int n_in = ms->n_in;
    const int nover = (int)n - n_in;
    int nbig = 0;
    for (int k = 0; k < ntop; k++) nbig += ms->top[k] < n_in;
    if (nover + nbig > kMaxMeshBig) {
        atomicOr(&st->status, (int32_t)ST_CAP_MESH);
        atomicMax((unsigned long long *)&st->required, (unsigned long long)(nover + nbig));
        ms->nbig = 0;
        return;
    }
    for (int k = 0; k < nover; k++) big[k] = n_in + k;
    nbig = nover;
    for (int k = 0; k < ntop; k++)
        if (ms->top[k] < n_in) big[nbig++] = ms->top[k];
    ms->nbig = nbig;
}

// One thread per moonlet of the mesh (sorted order): its neighbours (not among the
// all-pairs moonlets) in bucket order, then the all-pairs moonlets.  The three most
// massive only count their neighbours here; their sums come from k_mesh_big_sum.
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_gravity(DevState *st, MeshState *ms, const int4 *__restrict__ tab,
               const double4 *__restrict__ mpos, const int4 *__restrict__ mcell,
               const uint32_t *__restrict__ idx, const int32_t *__restrict__ big, int M,
               int count, double *__restrict__ ax, double *__restrict__ ay,
               double *__restrict__ az) {
    if (st->status & kSkipMask) return;
    const int64_t q = blockIdx.x * (int64_t)kMeshBlock + threadIdx.x;
    const int n_in = ms->n_in, stamp = ms->stamp, nbig = ms->nbig;
    const int t0 = ms->top[0], t1 = ms->top[1], t2 = ms->top[2];
    unsigned long long cnt = 0;
    if (q < n_in) {
        const double4 p = mpos[q];
        const int4 c = mcell[q];
        const bool top = q == t0 || q == t1 || q == t2;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int4 e = tab[bucket_of(c.x + dx, c.y + dy, c.z + dz, M)];
                    if (e.z != stamp) continue;
                    for (int r = e.x; r < e.y; r++) {
                        if (r == q) continue;
                        const int4 cr = mcell[r];
                        if (cr.x != c.x + dx || cr.y != c.y + dy || cr.z != c.z + dz) continue;
                        cnt++;
                        if (top || r == t0 || r == t1 || r == t2) continue;
                        add_pull(mpos[r], p.x, p.y, p.z, a0, a1, a2);
                    }
                }
        if (!top) {
            for (int k = 0; k < nbig; k++) {
                const int r = big[k];
                if (r != q) add_pull(mpos[r], p.x, p.y, p.z, a0, a1, a2);
            }
            const uint32_t i = idx[q];
            ax[i] = a0; ay[i] = a1; az[i] = a2;
        }
    }
    if (count) {
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        if ((threadIdx.x & (kWave - 1)) == 0 && cnt) atomicAdd(&ms->nbr_sum, cnt);
        if (q == 0) ms->measured = 1;
    }
}

// all-pairs sums of the big moonlets: block (chunk, row) sums a chunk of sources
// for big moonlets row, row + kMeshBigRows, ...
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_big_sum(const DevState *__restrict__ st, const MeshState *__restrict__ ms,
               const double4 *__restrict__ mpos, const int32_t *__restrict__ big, int64_t n,
               double *part) {
    __shared__ double red[3][kMeshBlock / kWave];
    if (st->status & kSkipMask) return;
    const int nbig = ms->nbig;
    const int64_t per = (n + kMeshChunks - 1) / kMeshChunks;
    const int64_t j0 = blockIdx.x * per;
    const int64_t j1 = j0 + per < n ? j0 + per : n;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = blockIdx.y; k < nbig; k += gridDim.y) {
        const int b = big[k];
        const double4 p = mpos[b];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kMeshBlock)
            if (j != b) add_pull(mpos[j], p.x, p.y, p.z, a0, a1, a2);
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o);
            a1 += __shfl_xor(a1, o);
            a2 += __shfl_xor(a2, o);
        }
        if (lane == 0) { red[0][w] = a0; red[1][w] = a1; red[2][w] = a2; }
        __syncthreads();
        if (threadIdx.x < 3) {
            double v = 0.0;
            for (int q = 0; q < kMeshBlock / kWave; q++) v += red[threadIdx.x][q];
            part[((int64_t)k * kMeshChunks + blockIdx.x) * 3 + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

__global__ void k_mesh_big_final(const DevState *__restrict__ st,
                                 const MeshState *__restrict__ ms, const int32_t *__restrict__ big,
                                 const uint32_t *__restrict__ idx, const double *__restrict__ part,
                                 double *ax, double *ay, double *az) {
    if (st->status & kSkipMask) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ms->nbig) return;
    double a[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < kMeshChunks; c++)
        for (int d = 0; d < 3; d++) a[d] += part[((int64_t)k * kMeshChunks + c) * 3 + d];
    const uint32_t i = idx[big[k]];
    ax[i] = a[0]; ay[i] = a[1]; az[i] = a[2];
}

// ------------------------------------------------------------------ collisions
__global__ void k_mesh_vel(const uint32_t *__restrict__ idx, const double *__restrict__ vx,
                           const double *__restrict__ vy, const double *__restrict__ vz,
                           const double *__restrict__ R, int64_t n, double4 *mvel) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) {
        const uint32_t i = idx[q];
        mvel[q] = make_double4(vx[i], vy[i], vz[i], R[i]);
    }
}

__global__ void k_mesh_col_init(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { st->npairs = 0; st->col_tests = 0; }
}

// one thread per moonlet of the mesh: its neighbours later in sorted order
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_collide(DevState *st, MeshState *ms, const int4 *__restrict__ tab,
               const double4 *__restrict__ mpos, const double4 *__restrict__ mvel,
               const int4 *__restrict__ mcell, const uint32_t *__restrict__ idx, int M, double dt,
               int count, int64_t *out, int64_t cap) {
    if (st->status & kSkipMask) return;
    const int64_t q = blockIdx.x * (int64_t)kMeshBlock + threadIdx.x;
    const int n_in = ms->n_in, stamp = ms->stamp;
    unsigned long long cnt = 0, tests = 0;
    if (q < n_in) {
        const double4 p = mpos[q], v = mvel[q];
        const int4 c = mcell[q];
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int4 e = tab[bucket_of(c.x + dx, c.y + dy, c.z + dz, M)];
                    if (e.z != stamp) continue;
                    for (int r = e.x; r < e.y; r++) {
                        if (r == q) continue;
                        const int4 cr = mcell[r];
                        if (cr.x != c.x + dx || cr.y != c.y + dy || cr.z != c.z + dz) continue;
                        cnt++;
                        if (r < q) continue;
                        const double4 pr = mpos[r], vr = mvel[r];
                        tests++;
                        if (pair_test(p.x, p.y, p.z, v.x, v.y, v.z, v.w, pr.x, pr.y, pr.z, vr.x,
                                      vr.y, vr.z, vr.w, dt))
                            record(out, cap, (unsigned long long *)&st->npairs, idx[q], idx[r]);
                    }
                }
    }
    for (int o = 32; o > 0; o >>= 1) {
        cnt += __shfl_xor(cnt, o);
        tests += __shfl_xor(tests, o);
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        if (tests) atomicAdd((unsigned long long *)&st->col_tests, tests);
        if (count && cnt) atomicAdd(&ms->nbr_sum, cnt);
    }
    if (count && q == 0) ms->measured = 1;
}

// the moonlets out of the mesh against every moonlet (each pair of two of them once)
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_collide_out(DevState *st, const MeshState *__restrict__ ms,
                   const double4 *__restrict__ mpos, const double4 *__restrict__ mvel,
                   const uint32_t *__restrict__ idx, int64_t n, double dt, int64_t *out,
                   int64_t cap) {
    if (st->status & kSkipMask) return;
    const int n_in = ms->n_in;
    const int nover = (int)n - n_in;
    if (nover > kMaxMeshBig) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            atomicOr(&st->status, (int32_t)ST_CAP_MESH);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)nover);
        }
        return;
    }
    const int64_t per = (n + kMeshChunks - 1) / kMeshChunks;
    const int64_t j0 = blockIdx.x * per;
    const int64_t j1 = j0 + per < n ? j0 + per : n;
    unsigned long long tests = 0;
    for (int k = blockIdx.y; k < nover; k += gridDim.y) {
        const int b = n_in + k;
        const double4 p = mpos[b], v = mvel[b];
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kMeshBlock) {
            if (j == b || (j >= n_in && j < b)) continue;
            const double4 pr = mpos[j], vr = mvel[j];
            tests++;
            if (pair_test(p.x, p.y, p.z, v.x, v.y, v.z, v.w, pr.x, pr.y, pr.z, vr.x, vr.y, vr.z,
                          vr.w, dt))
                record(out, cap, (unsigned long long *)&st->npairs, idx[b], idx[j]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) tests += __shfl_xor(tests, o);
    if ((threadIdx.x & (kWave - 1)) == 0 && tests)
        atomicAdd((unsigned long long *)&st->col_tests, tests);
}

int grid_of(int64_t n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

hipError_t launch_mesh_build(const Workspace &ws, const double *x, const double *y,
                             const double *z, const double *R, int64_t n, const ncorp_params &prm,
                             bool first, hipStream_t s) {
    const int M = ws.mesh_M;
    if (ws.clear_mesh)
        k_mesh_clear<<<4096, 256, 0, s>>>(ws.mtab, ws.mtab_n, ws.mesh);
    if (first && prm.mesh_gamma <= 0.0 && prm.mesh_rmax <= 0.0)
        k_mesh_rmax<<<1024, 256, 0, s>>>(x, y, z, n, ws.mesh);
    k_mesh_begin<<<1, 64, 0, s>>>(ws.mesh, ws.st, n, prm.mesh_neighbours, prm.mesh_aspect,
                                  prm.mesh_rmax, prm.mesh_gamma, prm.mesh_min_side / M);
    k_mesh_keys<<<grid_of(n, 256), 256, 0, s>>>(ws.st, ws.mesh, x, y, z, R, n, M, ws.mkeys,
                                                ws.midx);
    // key M^3 marks the moonlets out of the mesh; whole 16-bit digit pairs keep
    // the sorted result in mkeys / midx
    int bits = 1;
    while (bits < 62 && ((uint64_t)1 << bits) <= (uint64_t)M * M * M) bits++;
    bits = (bits + 15) / 16 * 16;
    bool in_b = false;
    hipError_t e = launch_radix_sort(ws.mkeys, ws.midx, ws.mkeys_alt, ws.midx_alt, n, bits,
                                     ws.hist, &in_b, s);
    if (e != hipSuccess) return e;
    if (in_b) return hipErrorInvalidValue;
    k_mesh_table<<<grid_of(n, 256), 256, 0, s>>>(ws.st, ws.mesh, ws.mkeys, ws.midx, x, y, z, n,
                                                 M, ws.mtab, ws.mpos, ws.mcell);
    return hipGetLastError();
}

hipError_t launch_mesh_gravity(const Workspace &ws, const double *m, double G, int64_t n,
                               bool count, double *ax, double *ay, double *az, hipStream_t s) {
    k_mesh_mu<<<grid_of(n, 256), 256, 0, s>>>(ws.midx, m, G, n, ws.mpos);
    k_mesh_top_part<<<kMeshTopBlocks, kMeshBlock, 0, s>>>(ws.st, m, ws.midx, n, ws.mtop_part);
    k_mesh_top_final<<<1, 64, 0, s>>>(ws.st, ws.mesh, m, ws.midx, n, ws.mtop_part, ws.mbig);
    k_mesh_gravity<<<grid_of(n, kMeshBlock), kMeshBlock, 0, s>>>(
        ws.st, ws.mesh, ws.mtab, ws.mpos, ws.mcell, ws.midx, ws.mbig, ws.mesh_M, count ? 1 : 0,
        ax, ay, az);
    k_mesh_big_sum<<<dim3(kMeshChunks, kMeshBigRows), kMeshBlock, 0, s>>>(ws.st, ws.mesh,
                                                                         ws.mpos, ws.mbig, n,
                                                                         ws.mbig_part);
    k_mesh_big_final<<<kMaxMeshBig / 256, 256, 0, s>>>(ws.st, ws.mesh, ws.mbig, ws.midx,
                                                      ws.mbig_part, ax, ay, az);
    return hipGetLastError();
}

hipError_t launch_mesh_collide(const Workspace &ws, const double *vx, const double *vy,
                               const double *vz, const double *R, int64_t n, double dt,
                               bool count, hipStream_t s) {
    k_mesh_vel<<<grid_of(n, 256), 256, 0, s>>>(ws.midx, vx, vy, vz, R, n, ws.mvel);
    k_mesh_col_init<<<1, 64, 0, s>>>(ws.st);
    k_mesh_collide<<<grid_of(n, kMeshBlock), kMeshBlock, 0, s>>>(
        ws.st, ws.mesh, ws.mtab, ws.mpos, ws.mvel, ws.mcell, ws.midx, ws.mesh_M, dt,
        count ? 1 : 0, ws.pairs_tmp, ws.pair_cap);
    k_mesh_collide_out<<<dim3(kMeshChunks, kMeshBigRows), kMeshBlock, 0, s>>>(
        ws.st, ws.mesh, ws.mpos, ws.mvel, ws.midx, n, dt, ws.pairs_tmp, ws.pair_cap);
    return hipGetLastError();
}

}  // namespace ncorp

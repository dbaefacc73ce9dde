// Brute-force module (Sect. 3.2): every pair of moonlets.  Gravity is the plain sum
//   a_i = sum_{j != i} G m_j (x_j - x_i) / |x_j - x_i|^3
// and the collision search tests every pair i < j with Eqs. (1)-(2).  Both work on
// the tree-ordered arrays of the last build (spatially sorted, which keeps each
// block's sources in cache) and write accelerations and pairs by input index.
//
// One thread per target, sources streamed through LDS in tiles shared by the block;
// FP64 throughout, each target's sum compensated (Neumaier) across tiles so that the
// O(N) terms of a large N add up without growing error.
#include "contact.h"

namespace ncorp {
namespace {

constexpr int kBruteBlock = 256;

__device__ __forceinline__ void neumaier(double &s, double &c, double v) {
    const double t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
}

__global__ void __launch_bounds__(kBruteBlock)
k_brute_gravity(const DevState *__restrict__ st, const double *__restrict__ xs,
                const double *__restrict__ ys, const double *__restrict__ zs,
                const double *__restrict__ mus, const uint32_t *__restrict__ idx, int64_t n,
                double *__restrict__ ax, double *__restrict__ ay, double *__restrict__ az) {
    __shared__ double4 tile[kBruteBlock];
    if (st->status & kSkipMask) return;
    const int64_t i = blockIdx.x * (int64_t)kBruteBlock + threadIdx.x;
    const bool live = i < n;
    const double x = live ? xs[i] : 0.0, y = live ? ys[i] : 0.0, z = live ? zs[i] : 0.0;
    double sx = 0.0, cx = 0.0, sy = 0.0, cy = 0.0, sz = 0.0, cz = 0.0;
    for (int64_t t0 = 0; t0 < n; t0 += kBruteBlock) {
        const int64_t j = t0 + threadIdx.x;
        __syncthreads();
        tile[threadIdx.x] = j < n ? make_double4(xs[j], ys[j], zs[j], mus[j])
                                  : make_double4(0.0, 0.0, 0.0, 0.0);
        __syncthreads();
        const int cnt = n - t0 < kBruteBlock ? (int)(n - t0) : kBruteBlock;
        // one tile summed plainly, then added to the compensated total
        double tx = 0.0, ty = 0.0, tz = 0.0;
        for (int k = 0; k < cnt; k++) {
            const double4 s = tile[k];
            const double dx = s.x - x, dy = s.y - y, dz = s.z - z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0 || t0 + k == i) continue;
            const double r = sqrt(r2);
            const double f = s.w / (r2 * r);
            tx += f * dx;
            ty += f * dy;
            tz += f * dz;
        }
        neumaier(sx, cx, tx);
        neumaier(sy, cy, ty);
        neumaier(sz, cz, tz);
    }
    if (live) {
        const uint32_t k = idx[i];
        ax[k] = sx + cx; ay[k] = sy + cy; az[k] = sz + cz;
    }
}

// every pair (i, j) of tree positions with i < j; recorded by input index
__global__ void __launch_bounds__(kBruteBlock)
k_brute_collide(DevState *st, const double *__restrict__ xs, const double *__restrict__ ys,
                const double *__restrict__ zs, const double *__restrict__ vxs,
                const double *__restrict__ vys, const double *__restrict__ vzs,
                const double *__restrict__ rads, const uint32_t *__restrict__ idx, int64_t n,
                double dt, int64_t *out, int64_t cap, unsigned long long *tests_part) {
    __shared__ double4 tp[kBruteBlock], tv[kBruteBlock];
    __shared__ unsigned long long red[kBruteBlock / kWave];
    if (st->status & kSkipMask) {
        if (threadIdx.x == 0) tests_part[blockIdx.x] = 0;
        return;
    }
    const int64_t i = blockIdx.x * (int64_t)kBruteBlock + threadIdx.x;
    const bool live = i < n;
    double4 p = make_double4(0.0, 0.0, 0.0, 0.0), v = p;
    if (live) {
        p = make_double4(xs[i], ys[i], zs[i], 0.0);
        v = make_double4(vxs[i], vys[i], vzs[i], rads[i]);
    }
    unsigned long long tests = 0;
    // sources after the block's first target only
    for (int64_t t0 = (int64_t)blockIdx.x * kBruteBlock; t0 < n; t0 += kBruteBlock) {
        const int64_t j = t0 + threadIdx.x;
        __syncthreads();
        if (j < n) {
            tp[threadIdx.x] = make_double4(xs[j], ys[j], zs[j], 0.0);
            tv[threadIdx.x] = make_double4(vxs[j], vys[j], vzs[j], rads[j]);
        }
        __syncthreads();
        const int cnt = n - t0 < kBruteBlock ? (int)(n - t0) : kBruteBlock;
        if (!live) continue;
        for (int k = 0; k < cnt; k++) {
            if (t0 + k <= i) continue;
            const double4 q = tp[k], w = tv[k];
            tests++;
            if (pair_test(p.x, p.y, p.z, v.x, v.y, v.z, v.w, q.x, q.y, q.z, w.x, w.y, w.z, w.w,
                          dt))
                record(out, cap, (unsigned long long *)&st->npairs, idx[i], idx[t0 + k]);
        }
    }
    for (int o = 32; o > 0; o >>= 1) tests += __shfl_xor(tests, o);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = tests;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < kBruteBlock / kWave; k++) t += red[k];
        tests_part[blockIdx.x] = t;
    }
}

}  // namespace

hipError_t launch_brute_gravity(const Workspace &ws, int64_t n, double *ax, double *ay,
                                double *az, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kBruteBlock - 1) / kBruteBlock;
    k_brute_gravity<<<(unsigned)blocks, kBruteBlock, 0, s>>>(ws.st, ws.xs, ws.ys, ws.zs, ws.mus,
                                                             ws.idx, n, ax, ay, az);
    return hipGetLastError();
}

hipError_t launch_brute_collide(const Workspace &ws, int64_t n, double dt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kBruteBlock - 1) / kBruteBlock;
    k_brute_collide<<<(unsigned)blocks, kBruteBlock, 0, s>>>(
        ws.st, ws.xs, ws.ys, ws.zs, ws.vxs, ws.vys, ws.vzs, ws.rads, ws.idx, n, dt, ws.pairs_tmp,
        ws.pair_cap, ws.count_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_u64(ws.count_part, blocks, (unsigned long long *)&ws.st->col_tests, true,
                          s);
}

}  // namespace ncorp

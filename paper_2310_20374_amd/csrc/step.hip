// Kick and drift of the leapfrog (Sect. 4.1) with the central mass computed
// exactly in the kick (App. B.1: a = -G M_c r / r^3; it is not part of the tree),
// optionally with the central body's J2 bulge and the quadrupolar tide of a distant
// body (App. B):
//   a_J2  = G M_c R^2 J2 / r^5 [ (15 z^2 - 3 r^2) / (2 r^2) r - 3 z e_z ]
//   a_sun = -G M_sun / a^3 ( r - 3 (r . r_sun) / a^2 r_sun ).
#include "ncorp_internal.h"

namespace ncorp {

__global__ void k_kick(double *__restrict__ vx, double *__restrict__ vy, double *__restrict__ vz,
                       const double *__restrict__ ax, const double *__restrict__ ay,
                       const double *__restrict__ az, const double *__restrict__ x,
                       const double *__restrict__ y, const double *__restrict__ z, int64_t n,
                       double h, CentralBody b, const double *__restrict__ R,
                       double4 *__restrict__ pack, const double4 *__restrict__ acc4) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double px = x[i], py = y[i], pz = z[i];
        const double r2 = px * px + py * py + pz * pz;
        const double r = sqrt(r2);
        const double f = -b.GM / (r2 * r);
        double gx = f * px, gy = f * py, gz = f * pz;
        if (b.GMR2J2 != 0.0) {
            const double c = b.GMR2J2 / (r2 * r2 * r);
            const double k = (15.0 * pz * pz - 3.0 * r2) / (2.0 * r2);
            gx += c * (k * px);
            gy += c * (k * py);
            gz += c * (k * pz - 3.0 * pz);
        }
        if (b.GMsun != 0.0) {
            const double q = 3.0 * (px * b.sx + py * b.sy + pz * b.sz) / b.a2;
            const double g = -b.GMsun / b.a3;
            gx += g * (px - q * b.sx);
            gy += g * (py - q * b.sy);
            gz += g * (pz - q * b.sz);
        }
        if (acc4) {
            const double4 a = acc4[i];
            gx += a.x; gy += a.y; gz += a.z;
        } else if (ax) {
            gx += ax[i]; gy += ay[i]; gz += az[i];
        }
        const double ux = vx[i] + h * gx, uy = vy[i] + h * gy, uz = vz[i] + h * gz;
        vx[i] = ux;
        vy[i] = uy;
        vz[i] = uz;
        // the (v, R) record the next collision search gathers into tree order
        if (pack) pack[i] = make_double4(ux, uy, uz, R[i]);
    }
}

__global__ void k_drift(double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
                        const double *__restrict__ vx, const double *__restrict__ vy,
                        const double *__restrict__ vz, int64_t n, double dt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += dt * vx[i];
        y[i] += dt * vy[i];
        z[i] += dt * vz[i];
    }
}

// The drift of a step whose next build takes its root cube from the new positions:
// also their largest |coordinate| (bit patterns of the non-negative values, so the
// integer maximum is the value's; non-finite coordinates latched), the same word the
// key pass of a plain build forms.  Few blocks, four moonlets per thread and round,
// one atomic per block on the word.
__global__ void k_drift_max(double *__restrict__ x, double *__restrict__ y,
                            double *__restrict__ z, const double *__restrict__ vx,
                            const double *__restrict__ vy, const double *__restrict__ vz,
                            int64_t n, double dt, DevState *st) {
    __shared__ unsigned long long red[256 / kWave];
    constexpr int kBatch = 4;
    unsigned long long m = 0ull;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n;
         i0 += kBatch * stride) {
        double p[kBatch][3];
#pragma unroll
        for (int b = 0; b < kBatch; b++) {
            const int64_t i = i0 + b * stride;
            if (i < n) {
                p[b][0] = x[i] + dt * vx[i];
                p[b][1] = y[i] + dt * vy[i];
                p[b][2] = z[i] + dt * vz[i];
            }
        }
#pragma unroll
        for (int b = 0; b < kBatch; b++) {
            const int64_t i = i0 + b * stride;
            if (i >= n) continue;
            x[i] = p[b][0];
            y[i] = p[b][1];
            z[i] = p[b][2];
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double a = fabs(p[b][k]);
                if (!(a <= 1.79769313486231570e308)) { bad = true; continue; }
                const unsigned long long u = (unsigned long long)__double_as_longlong(a);
                m = u > m ? u : m;
            }
        }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) red[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); k++) m = red[k] > m ? red[k] : m;
        atomicMax((unsigned long long *)&st->max_abs, m);
    }
    if (__any(bad) && l == 0) atomicOr(&st->status, (int32_t)ST_NONFINITE);
}

static int grid1(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t launch_kick(double *vx, double *vy, double *vz, const double *ax, const double *ay,
                       const double *az, const double *x, const double *y, const double *z,
                       int64_t n, double h, const CentralBody &b, const double *R,
                       double4 *pack, hipStream_t s, const double4 *acc4) {
    k_kick<<<grid1(n), 256, 0, s>>>(vx, vy, vz, ax, ay, az, x, y, z, n, h, b, R, pack, acc4);
    return hipGetLastError();
}

hipError_t launch_drift(double *x, double *y, double *z, const double *vx, const double *vy,
                        const double *vz, int64_t n, double dt, hipStream_t s, DevState *st) {
    if (st) {
        const int64_t g = (n + 255) / 256;
        k_drift_max<<<(int)(g > 256 ? 256 : g), 256, 0, s>>>(x, y, z, vx, vy, vz, n, dt, st);
    } else {
        k_drift<<<grid1(n), 256, 0, s>>>(x, y, z, vx, vy, vz, n, dt);
    }
    return hipGetLastError();
}

}  // namespace ncorp

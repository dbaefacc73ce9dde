// The pair test of Sect. 3.1 and the recording of colliding pairs, shared by the
// tree and mesh collision searches:
//   Delta = (dr.dv)^2 + dv^2 [(R1 + R2)^2 - dr^2]                      (Eq. 1)
//   dt_c  = -(dr.dv + sqrt(Delta)) / dv^2, collision iff 0 <= dt_c <= dt (Eq. 2)
// FP64 with a fixed operation order and no contraction, symmetric under swapping
// the two moonlets bit for bit (dr and dv only change sign).
#pragma once

#include "ncorp_internal.h"

namespace ncorp {

// contact time dt_c of Eq. (2) when 0 <= dt_c <= dt, else -1
__device__ __forceinline__ double contact_time(double x1, double y1, double z1, double vx1,
                                               double vy1, double vz1, double R1, double x2,
                                               double y2, double z2, double vx2, double vy2,
                                               double vz2, double R2, double dt) {
    double dx = x1 - x2, dy = y1 - y2, dz = z1 - z2;
    double dvx = vx1 - vx2, dvy = vy1 - vy2, dvz = vz1 - vz2;
    double rv = dx * dvx + dy * dvy + dz * dvz;
    double v2 = dvx * dvx + dvy * dvy + dvz * dvz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double Rs = R1 + R2;
    double disc = rv * rv + v2 * (Rs * Rs - r2);
    if (!(v2 > 0.0) || !(disc >= 0.0)) return -1.0;
    double tc = -(rv + sqrt(disc)) / v2;
    return (tc >= 0.0 && tc <= dt) ? tc : -1.0;
}

__device__ __forceinline__ bool pair_test(double x1, double y1, double z1, double vx1,
                                          double vy1, double vz1, double R1, double x2,
                                          double y2, double z2, double vx2, double vy2,
                                          double vz2, double R2, double dt) {
    return contact_time(x1, y1, z1, vx1, vy1, vz1, R1, x2, y2, z2, vx2, vy2, vz2, R2, dt) >= 0.0;
}

__device__ __forceinline__ void record(int64_t *out, int64_t cap, unsigned long long *count,
                                       uint32_t ia, uint32_t ib) {
    uint32_t lo = ia < ib ? ia : ib, hi = ia < ib ? ib : ia;
    unsigned long long k = atomicAdd(count, 1ull);
    if ((int64_t)k < cap) out[k] = ((int64_t)lo << 32) | (int64_t)hi;
}

}  // namespace ncorp

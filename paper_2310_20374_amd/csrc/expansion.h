// Derivative tensors of 1/|R| and their contraction with scaled multipole moments,
// shared by the M2L kernel (Eq. 25) and the standard tree code's cell-moonlet terms.
//
// D comes from the recurrence of McMurchie & Davidson (J. Comput. Phys. 26, 1978)
// written for 1/r: with R^n_000 = (-1)^n (2n-1)!! r^-(2n+1),
//   R^n_{a+1,b,c} = a R^{n+1}_{a-1,b,c} + x R^{n+1}_{a,b,c}  (same for y, z),
// and D_{abc} = R^0_{abc}.
#pragma once

#include "ncorp_internal.h"

namespace ncorp {

template <int P, typename T>
__device__ __forceinline__ void green_derivs(T x, T y, T z, T rinv, T *D) {
    const T rinv2 = rinv * rinv;
    T g[P + 1];
    g[0] = rinv;
#pragma unroll
    for (int n = 1; n <= P; n++) g[n] = -(T)(2 * n - 1) * rinv2 * g[n - 1];
    // level n overwrites level n+1 in place: orders are visited from high to low,
    // so every value still needed (orders k-1, k-2 of level n+1) is intact
    D[0] = g[P];
#pragma unroll
    for (int n = P - 1; n >= 0; n--) {
#pragma unroll
        for (int k = P - n; k >= 1; k--)
#pragma unroll
            for (int b = 0; b <= k; b++)
#pragma unroll
                for (int c = 0; c <= k - b; c++) {
                    const int a = k - b - c;
                    T v;
                    if (a > 0) {
                        v = x * D[sidx(a - 1, b, c)];
                        if (a > 1) v += (T)(a - 1) * D[sidx(a - 2, b, c)];
                    } else if (b > 0) {
                        v = y * D[sidx(a, b - 1, c)];
                        if (b > 1) v += (T)(b - 1) * D[sidx(a, b - 2, c)];
                    } else {
                        v = z * D[sidx(a, b, c - 1)];
                        if (c > 1) v += (T)(c - 1) * D[sidx(a, b, c - 2)];
                    }
                    D[sidx(a, b, c)] = v;
                }
        D[0] = g[n];
    }
}

template <typename T> __device__ __forceinline__ T rsqrt_t(T v);
template <> __device__ __forceinline__ double rsqrt_t<double>(double v) { return 1.0 / sqrt(v); }
template <> __device__ __forceinline__ float rsqrt_t<float>(float v) { return rsqrtf(v); }

template <typename T> __device__ __forceinline__ T fma_t(T a, T b, T c);
template <> __device__ __forceinline__ double fma_t<double>(double a, double b, double c) {
    return fma(a, b, c);
}
template <> __device__ __forceinline__ float fma_t<float>(float a, float b, float c) {
    return fmaf(a, b, c);
}

// acc_a += sum_{b} sign(|b|) D_{a+b} Mt_b over the Eq. (25) index ranges, for
// the output orders MLO..MHI only (acc indexed from cidx(MLO, 0, 0))
template <int P, int MLO, int MHI, typename T>
__device__ __forceinline__ void m2l_contract(const T *D, const T *__restrict__ mb, T *acc) {
    constexpr int base = cidx(MLO, 0, 0);
#pragma unroll
    for (int n = 0; n <= P - MLO; n++) {
        if (n == 1) continue;
#pragma unroll
        for (int b2 = 0; b2 <= n; b2++)
#pragma unroll
            for (int c2 = 0; c2 <= n - b2; c2++) {
                const int a2 = n - b2 - c2;
                const T mt = mb[midx(a2, b2, c2)];
                const T mv = (n & 1) ? -mt : mt;
#pragma unroll
                for (int m = MLO; m <= (MHI < P - n ? MHI : P - n); m++)
#pragma unroll
                    for (int b = 0; b <= m; b++)
#pragma unroll
                        for (int c = 0; c <= m - b; c++) {
                            const int a = m - b - c;
                            acc[cidx(a, b, c) - base] = fma_t<T>(
                                D[sidx(a + a2, b + b2, c + c2)], mv, acc[cidx(a, b, c) - base]);
                        }
            }
    }
}

}  // namespace ncorp

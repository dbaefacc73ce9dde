// Interaction tensors (Eq. 25) for every well-separated pair found by the walk.
//
// Target-major: one wave per target cell A, lanes over A's sources B (grouped and
// sorted by the list builder), each lane accumulating
//   C^(m)_a(s_A) += sum_{n=0, n!=1}^{p-m} (-1)^n sum_{|b|=n} D_{a+b}(R) Mt_b(B),
// with R = s_A - s_B, D_g = d^g (1/|R|) and Mt_b = M_b / b! (the n! of Eq. 25 and
// the multinomial weights of the symmetric inner product cancel into 1/b!).  The
// wave then sums its 64 partial tensors order by order through LDS.  Both
// directions of a pair are separate entries of the list, so every target's sum has
// a fixed order and the result does not depend on scheduling.  D and the
// contraction are in expansion.h.
#include "ncorp_internal.h"
#include "expansion.h"

namespace ncorp {

constexpr int kM2LBlock = 64;     // one wave per block, one target per wave

// FP64 at high order splits the output orders over passes (D is recomputed per
// pass) so that the accumulators and D stay in registers.
template <int P, typename T> struct M2LSplit { static constexpr int K1 = P, K2 = P; };
template <> struct M2LSplit<6, double> { static constexpr int K1 = 4, K2 = 5; };
template <> struct M2LSplit<5, double> { static constexpr int K1 = 3, K2 = 5; };

// Components of C staged per round of the wave sum when one pass covers every order:
// half of them, so the buffer (and the occupancy it limits) is half as large.
template <int P> constexpr int red_chunk() { return (n_local(P) + 1) / 2; }

// Row stride (elements) of the wave-sum buffer: one round's components when one pass
// covers every order, else one order; odd, so a lane's row and a column are both free
// of bank conflicts.
template <int P, typename T> constexpr int red_stride() {
    return (M2LSplit<P, T>::K1 == P ? red_chunk<P>() : ncomp(P)) | 1;
}

// one pass over a target's sources for the output orders MLO..MHI
template <int P, int MLO, int MHI, typename T>
__device__ __forceinline__ void m2l_pass(const double4 gA, const double4 *__restrict__ gcell,
                                         const T *__restrict__ mult,
                                         const int32_t *__restrict__ srcs, int len, double *out,
                                         T *red) {
    constexpr int RS = red_stride<P, T>();
    constexpr int NM = n_mult(P), ND = off_order(P + 1);
    constexpr int NA = cidx(MHI + 1, 0, 0) - cidx(MLO, 0, 0);
    const int lane = threadIdx.x;
    T acc[NA];
#pragma unroll
    for (int k = 0; k < NA; k++) acc[k] = (T)0;
    for (int i = lane; i < len; i += kWave) {
        const int B = srcs[i];
        const double4 gB = gcell[B];
        const T x = (T)(gA.x - gB.x), y = (T)(gA.y - gB.y), z = (T)(gA.z - gB.z);
        const T r2 = x * x + y * y + z * z;
        T D[ND];
        green_derivs<P, T>(x, y, z, rsqrt_t<T>(r2), D);
        m2l_contract<P, MLO, MHI, T>(D, mult + (int64_t)B * NM, acc);
    }
    // wave sum of every component in lane order (FP64)
    if constexpr (MLO == 1 && MHI == P && M2LSplit<P, T>::K1 == P) {
        // all orders at once, in two rounds of CH components: lane k sums component
        // c0 + k of the round
        constexpr int CH = red_chunk<P>();
#pragma unroll
        for (int c0 = 0; c0 < NA; c0 += CH) {
#pragma unroll
            for (int k = 0; k < CH; k++)
                if (c0 + k < NA) red[lane * RS + k] = acc[c0 + k];
            __syncthreads();
            const int nk = NA - c0 < CH ? NA - c0 : CH;
            for (int k = lane; k < nk; k += kWave) {
                double s = 0.0;
                for (int l = 0; l < kWave; l++) s += (double)red[l * RS + k];
                out[cidx(MLO, 0, 0) + c0 + k] = s;
            }
            __syncthreads();
        }
    } else {
#pragma unroll
        for (int m = MLO; m <= MHI; m++) {
            const int base = cidx(m, 0, 0) - cidx(MLO, 0, 0);
#pragma unroll
            for (int k = 0; k < ncomp(m); k++) red[lane * RS + k] = acc[base + k];
            __syncthreads();
            if (lane < ncomp(m)) {
                double s = 0.0;
                for (int l = 0; l < kWave; l++) s += (double)red[l * RS + lane];
                out[cidx(m, 0, 0) + lane] = s;
            }
            __syncthreads();
        }
    }
}

// LDS of the wave-sum buffer, in ints: a target's list is sorted there first
template <int P, typename T> constexpr int red_ints() {
    return (int)(sizeof(T) * kWave * red_stride<P, T>() / 4) & ~3;
}

template <int P, typename T>
__global__ void __launch_bounds__(kM2LBlock, 2)
k_m2l(const DevState *__restrict__ st, const double4 *__restrict__ gcell,
      const T *__restrict__ mult, const int32_t *__restrict__ cnt, int32_t *__restrict__ seg,
      int stride, double *__restrict__ local) {
    constexpr int NL = n_local(P);
    constexpr int K1 = M2LSplit<P, T>::K1, K2 = M2LSplit<P, T>::K2;
    __shared__ __align__(16) T red[kWave * red_stride<P, T>()];
    __shared__ int32_t s_list[kM2LListLDS];
    extern __shared__ __align__(16) int32_t dyn[];   // sort scratch if red is too small
    if (st->status & kSkipMask) return;
    const int need = ((stride < kM2LListLDS ? stride : kM2LListLDS) + 3) & ~3;
    int32_t *scratch = need <= red_ints<P, T>() ? (int32_t *)red : dyn;
    const int nc = st->ncells;
    const int lane = threadIdx.x;
    for (int A = blockIdx.x; A < nc; A += gridDim.x) {
        const int len = cnt[A];
        double *out = local + (int64_t)A * NL;
        if (len == 0) {
            for (int k = lane; k < NL; k += kWave) out[k] = 0.0;
            continue;
        }
        int32_t *list = seg + (int64_t)A * stride;
        const int32_t *srcs = list;
        if (len <= kM2LListLDS) {
            // usual case: sorted copy in LDS
            const int len4 = (len + 3) & ~3;
            for (int i = lane; i < len4; i += kWave) scratch[i] = i < len ? list[i] : 0x7fffffff;
            __syncthreads();
            const int4 *s4 = reinterpret_cast<const int4 *>(scratch);
            for (int i = lane; i < len; i += kWave) {
                const int v = scratch[i];
                int r = 0;
                #pragma unroll 8
                for (int j = 0; j < len4 / 4; j++) {
                    const int4 t = s4[j];
                    r += (t.x < v) + (t.y < v) + (t.z < v) + (t.w < v);
                }
                s_list[r] = v;
            }
            __syncthreads();
            srcs = s_list;
        }                                       // longer lists: sorted by the pre-pass
        const double4 gA = gcell[A];
        m2l_pass<P, 1, K1, T>(gA, gcell, mult, srcs, len, out, red);
        if (K2 > K1) m2l_pass<P, (K1 < P ? K1 + 1 : P), K2, T>(gA, gcell, mult, srcs, len, out, red);
        if (P > K2) m2l_pass<P, (K2 < P ? K2 + 1 : P), P, T>(gA, gcell, mult, srcs, len, out, red);
    }
}

template <int P, typename T>
static void launch_m2l_t(const Workspace &ws, const T *mult, hipStream_t s) {
    int g = (int)(ws.cell_cap < 16384 ? ws.cell_cap : 16384);
    if (g < 1) g = 1;
    const int s4 = ((ws.m2l_stride < kM2LListLDS ? ws.m2l_stride : kM2LListLDS) + 3) & ~3;
    const size_t dyn = s4 <= red_ints<P, T>() ? 0 : (size_t)s4 * sizeof(int32_t);
    k_m2l<P, T><<<g, kM2LBlock, dyn, s>>>(ws.st, ws.gcell, mult, ws.m2l_cnt, ws.m2l_seg,
                                          ws.m2l_stride, ws.local);
}

template <int P>
static void launch_m2l_p(const Workspace &ws, int precision, hipStream_t s) {
    if (precision == NCORP_FP32_BULK) launch_m2l_t<P, float>(ws, ws.mult32, s);
    else launch_m2l_t<P, double>(ws, ws.mult, s);
}

hipError_t launch_m2l(const Workspace &ws, int p, int precision, hipStream_t s) {
    switch (p) {
        case 1: launch_m2l_p<1>(ws, precision, s); break;
        case 2: launch_m2l_p<2>(ws, precision, s); break;
        case 3: launch_m2l_p<3>(ws, precision, s); break;
        case 4: launch_m2l_p<4>(ws, precision, s); break;
        case 5: launch_m2l_p<5>(ws, precision, s); break;
        case 6: launch_m2l_p<6>(ws, precision, s); break;
        default: break;
    }
    return hipGetLastError();
}

}  // namespace ncorp

// Device-wide exclusive scan of int32 counts whose length lives in device memory
// (so it can be enqueued without a host round trip): reduce per segment, scan the
// segment totals in one block, rescan each segment with its carry.
#include "ncorp_internal.h"

namespace ncorp {

constexpr int kScanBlock = 1024;
constexpr int kScanMaxGrid = 1024;

__device__ __forceinline__ int32_t block_incl_scan(int32_t v, int32_t *sh) {
    // sh: at least kScanBlock / 64 entries
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t t = __shfl_up(x, o);
        if (lane >= o) x += t;
    }
    if (lane == kWave - 1) sh[w] = x;
    __syncthreads();
    if (w == 0) {
        int nw = blockDim.x / kWave;
        int32_t y = lane < nw ? sh[lane] : 0;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            int32_t t = __shfl_up(y, o);
            if (lane >= o) y += t;
        }
        if (lane < nw) sh[lane] = y;
    }
    __syncthreads();
    int32_t r = x + (w > 0 ? sh[w - 1] : 0);
    __syncthreads();
    return r;
}

static __device__ __forceinline__ void seg_bounds(int64_t n, int64_t &seg) {
    int64_t g = gridDim.x;
    seg = (n + g - 1) / g;
    seg = (seg + kScanBlock - 1) / kScanBlock * kScanBlock;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_reduce(const int32_t *__restrict__ in, const int32_t *n_dev, int32_t *partials) {
    __shared__ int32_t sh[kScanBlock / kWave];
    int64_t n = *n_dev, seg;
    seg_bounds(n, seg);
    int64_t b0 = (int64_t)blockIdx.x * seg, b1 = b0 + seg < n ? b0 + seg : n;
    int32_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kScanBlock) s += in[i];
    // block reduce
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int k = 0; k < kScanBlock / kWave; k++) t += sh[k];
        partials[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_partials(int32_t *partials, int g, int32_t *total_dev) {
    __shared__ int32_t sh[kScanBlock / kWave];
    int32_t v = threadIdx.x < g ? partials[threadIdx.x] : 0;
    int32_t incl = block_incl_scan(v, sh);
    if (threadIdx.x < g) partials[threadIdx.x] = incl - v;
    if (threadIdx.x == kScanBlock - 1) *total_dev = incl;
}

__global__ void __launch_bounds__(kScanBlock)
k_scan_apply(const int32_t *in, int32_t *out, const int32_t *n_dev,
             const int32_t *__restrict__ partials) {
    __shared__ int32_t sh[kScanBlock / kWave];
    int64_t n = *n_dev, seg;
    seg_bounds(n, seg);
    int64_t b0 = (int64_t)blockIdx.x * seg, b1 = b0 + seg < n ? b0 + seg : n;
    int32_t carry = partials[blockIdx.x];
    for (int64_t t0 = b0; t0 < b1; t0 += kScanBlock) {
        int64_t i = t0 + threadIdx.x;
        int32_t v = i < b1 ? in[i] : 0;
        int32_t incl = block_incl_scan(v, sh);
        if (i < b1) out[i] = carry + incl - v;
        __shared__ int32_t last;
        if (threadIdx.x == kScanBlock - 1) last = incl;
        __syncthreads();
        carry += last;
        __syncthreads();
    }
}

hipError_t launch_scan(const int32_t *in, int32_t *out, const int32_t *n_dev, int64_t n_cap,
                       int32_t *partials, int32_t *total_dev, hipStream_t s) {
    int64_t g = (n_cap + kScanBlock * 4 - 1) / (kScanBlock * 4);
    if (g < 1) g = 1;
    if (g > kScanMaxGrid) g = kScanMaxGrid;
    k_scan_reduce<<<(int)g, kScanBlock, 0, s>>>(in, n_dev, partials);
    k_scan_partials<<<1, kScanBlock, 0, s>>>(partials, (int)g, total_dev);
    k_scan_apply<<<(int)g, kScanBlock, 0, s>>>(in, out, n_dev, partials);
    return hipGetLastError();
}

}  // namespace ncorp

// Root cube, 63-bit Hilbert keys and the stable radix sort that puts the moonlets
// in Hilbert order (Sect. 3.4.6).  All three are bandwidth-bound streaming passes.
#include "ncorp_internal.h"

namespace ncorp {

// ------------------------------------------------------------------ helpers
__global__ void k_reset_state(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        DevState z{};
        // the bucket sort's boundaries for the next build outlive a fresh build
        z.bs_L = st->bs_L;
        z.bs_valid = st->bs_valid;
        z.bs_n = st->bs_n;
        z.bs_sub_wr = st->bs_sub_wr;
        *st = z;
    }
}

hipError_t launch_reset_state(const Workspace &ws, hipStream_t s) {
    k_reset_state<<<1, 64, 0, s>>>(ws.st);
    return hipGetLastError();
}


__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t *p, int64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int grid_for(int64_t n, int block, int cap = 4096) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i64<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ root cube
// max |coordinate| over finite values; non-finite coordinates latch a status bit.
// Non-negative doubles order like their bit patterns, so an unsigned 64-bit
// atomic max gives the maximum.
__global__ void k_max_abs(const double *__restrict__ x, const double *__restrict__ y,
                          const double *__restrict__ z, int64_t n, DevState *st) {
    __shared__ unsigned long long red[256 / kWave];
    unsigned long long m = 0ull;
    bool bad = false;
    // four strided moonlets per round, their loads issued together
    constexpr int kBatch = 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n;
         i0 += kBatch * stride) {
        double v[kBatch][3];
#pragma unroll
        for (int b = 0; b < kBatch; b++) {
            const int64_t i = i0 + b * stride;
            const bool in = i < n;
            v[b][0] = in ? x[i] : 0.0;
            v[b][1] = in ? y[i] : 0.0;
            v[b][2] = in ? z[i] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < kBatch; b++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                const double a = fabs(v[b][k]);
                if (!(a <= 1.79769313486231570e308)) { bad = true; continue; }
                const unsigned long long u = (unsigned long long)__double_as_longlong(a);
                m = u > m ? u : m;
            }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        unsigned long long t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) red[w] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); k++) m = red[k] > m ? red[k] : m;
        atomicMax((unsigned long long *)&st->max_abs, m);
    }
    if (__any(bad) && l == 0) atomicOr(&st->status, (int32_t)ST_NONFINITE);
}

// Batched calls: block d writes the disk id d over moonlets [off[d], off[d+1]) and
// clears the disk's running max; the offsets are checked on the way (non-decreasing,
// from 0 to n), a violation latches ST_BAD_OFFSETS and every later pass of the call
// does nothing.  Ids stay below NCORP_MAX_DISKS whatever the offsets hold.
__global__ void k_disk_ids(const int64_t *__restrict__ off, int nd, int64_t n,
                           uint16_t *__restrict__ seg, unsigned long long *__restrict__ disk_max,
                           DevState *st) {
    for (int d = blockIdx.x; d < nd; d += gridDim.x) {
        const int64_t a = off[d], b = off[d + 1];
        if (threadIdx.x == 0) {
            disk_max[d] = 0ull;
            const bool bad = a > b || a < 0 || b > n || (d == 0 && a != 0) ||
                             (d == nd - 1 && b != n);
            if (bad) atomicOr(&st->status, (int32_t)ST_BAD_OFFSETS);
        }
        const int64_t lo = a < 0 ? 0 : (a > n ? n : a);
        const int64_t hi = b < lo ? lo : (b > n ? n : b);
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) seg[i] = (uint16_t)d;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->ndisks = nd;
}

// max |coordinate| per disk.  Every wave scans one contiguous chunk of moonlets in
// coalesced rounds of 64; each lane keeps a running max for the disk it is in and
// publishes it (one atomic) only when it enters another disk, and at the end the
// wave reduces first if all its lanes ended in the same disk.
__global__ void k_max_abs_seg(const double *__restrict__ x, const double *__restrict__ y,
                              const double *__restrict__ z, int64_t n,
                              const uint16_t *__restrict__ seg,
                              unsigned long long *__restrict__ disk_max, DevState *st) {
    const int lane = threadIdx.x % kWave;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    const int64_t w = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    const int64_t chunk = ((n + nw - 1) / nw + kWave - 1) / kWave * kWave;
    const int64_t b0 = w * chunk;
    const int64_t b1 = b0 + chunk < n ? b0 + chunk : n;
    bool bad = false;
    int cur = -1;
    unsigned long long run = 0ull;
    for (int64_t b = b0; b < b1; b += kWave) {
        const int64_t i = b + lane;
        if (i >= b1) continue;
        const int d = seg[i];
        if (d != cur) {
            if (cur >= 0) atomicMax(&disk_max[cur], run);
            cur = d;
            run = 0ull;
        }
        double v[3] = {x[i], y[i], z[i]};
#pragma unroll
        for (int k = 0; k < 3; k++) {
            double a = fabs(v[k]);
            if (!(a <= 1.79769313486231570e308)) { bad = true; continue; }
            unsigned long long u = (unsigned long long)__double_as_longlong(a);
            run = u > run ? u : run;
        }
    }
    const int c0 = __shfl(cur, 0);
    if (__all(cur == c0)) {
        for (int o = kWave / 2; o > 0; o >>= 1) {
            unsigned long long t = __shfl_xor(run, o);
            run = t > run ? t : run;
        }
        if (lane == 0 && c0 >= 0) atomicMax(&disk_max[c0], run);
    } else if (cur >= 0) {
        atomicMax(&disk_max[cur], run);
    }
    if (__any(bad) && lane == 0) atomicOr(&st->status, (int32_t)ST_NONFINITE);
}

// ------------------------------------------------------------------ keys
// q = floor((x + L) * 2^20 / L), clamped to [0, 2^21 - 1]; with L a power of two the
// scale is exact, so the result depends only on the correctly rounded x + L.
__device__ __forceinline__ uint32_t quantize(double x, double L, double scale) {
    double t = (x + L) * scale;
    if (!(t >= 0.0)) return 0u;
    if (t >= 2097152.0) return 2097151u;
    uint32_t q = (uint32_t)floor(t);
    return q > 2097151u ? 2097151u : q;
}

// 3-D Hilbert index of (q0, q1, q2), 21 bits each, in Skilling's transpose form
// (AIP Conf. Proc. 707, 2004): per level, invert or exchange the lower bits, then
// Gray-code the axes; the index interleaves the transposed bits x, y, z from the
// most significant level down.
__device__ __forceinline__ uint64_t hilbert21(uint32_t q0, uint32_t q1, uint32_t q2) {
    uint32_t X[3] = {q0, q1, q2};
#pragma unroll
    for (int lv = 20; lv >= 1; lv--) {
        uint32_t Q = 1u << lv, P = Q - 1u;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
#pragma unroll
    for (int lv = 20; lv >= 1; lv--)
        if (X[2] & (1u << lv)) t ^= (1u << lv) - 1u;
    X[0] ^= t; X[1] ^= t; X[2] ^= t;
    // interleave: bit b of axis i lands at position 3b + (2 - i)
    uint64_t h = 0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        uint64_t v = X[i];
        // spread 21 bits to every third position
        v = (v | (v << 32)) & 0x1f00000000ffffull;
        v = (v | (v << 16)) & 0x1f0000ff0000ffull;
        v = (v | (v << 8)) & 0x100f00f00f00f00full;
        v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
        v = (v | (v << 2)) & 0x1249249249249249ull;
        h |= v << (2 - i);
    }
    return h;
}

// smallest power of two strictly above mx (1 when every coordinate is 0)
__device__ __forceinline__ double root_half_width(unsigned long long mx_bits) {
    const double mx = __longlong_as_double((long long)mx_bits);
    if (!(mx > 0.0)) return 1.0;
    int e;
    frexp(mx, &e);           // mx = f 2^e, 0.5 <= f < 1
    return ldexp(1.0, e);
}

// Keys of every moonlet against the root cube of its disk (seg == nullptr: one
// disk).  mx: per-disk max |coordinate| bit patterns; fixed_L > 0 overrides them.
// Also records each disk's half-width in disk_L (and disk 0's in st->L).
__global__ void k_keys(const double *__restrict__ x, const double *__restrict__ y,
                       const double *__restrict__ z, int64_t n, double fixed_L,
                       const unsigned long long *__restrict__ mx,
                       const uint16_t *__restrict__ seg, int nd, double *__restrict__ disk_L,
                       DevState *st, uint64_t *__restrict__ keys, uint32_t *__restrict__ idx,
                       double4 *__restrict__ pack4, const double *__restrict__ m, double G) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid < nd) {
        const double L = fixed_L > 0.0 ? fixed_L : root_half_width(mx[gid]);
        disk_L[gid] = L;
        if (gid == 0) st->L = L;
    }
    double L = fixed_L > 0.0 ? fixed_L : root_half_width(mx[0]);
    for (int64_t i = gid; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (seg && !(fixed_L > 0.0)) L = root_half_width(mx[seg[i]]);
        const double scale = 1048576.0 / L;
        const double px = x[i], py = y[i], pz = z[i];
        keys[i] = hilbert21(quantize(px, L, scale), quantize(py, L, scale),
                            quantize(pz, L, scale));
        idx[i] = (uint32_t)i;
        // one record per moonlet for the gather (with G m when the caller has the masses)
        pack4[i] = make_double4(px, py, pz, m ? G * m[i] : 0.0);
    }
}

// radix passes of a build: 8 over the 63-bit keys, then (batched calls) 1 or 2 over
// the disk id, the most significant digit
static int disk_passes(int nd) { return nd <= 1 ? 0 : (nd <= 256 ? 1 : 2); }

hipError_t launch_keys(const Workspace &ws, const double *x, const double *y,
                       const double *z, int64_t n, double root_half_width,
                       const int64_t *disk_off, const double *m, double G, hipStream_t s,
                       bool max_ready) {
    // the sort ends in ws.keys / ws.idx: the bucket sort and an odd number of radix
    // passes start in the other buffers
    const bool odd = bucket_sort_applies(ws, n) || (8 + disk_passes(ws.ndisks)) % 2 == 1;
    uint64_t *kout = odd ? ws.keys_alt : ws.keys;
    uint32_t *vout = odd ? ws.idx_alt : ws.idx;
    if (disk_off) {
        const int nd = ws.ndisks;
        k_disk_ids<<<nd < 4096 ? nd : 4096, 256, 0, s>>>(disk_off, nd, n, ws.seg, ws.disk_max,
                                                         ws.st);
        // also run with a fixed root: it latches non-finite coordinates
        k_max_abs_seg<<<grid_for(n, 256, 512), 256, 0, s>>>(x, y, z, n, ws.seg, ws.disk_max,
                                                            ws.st);
        const int64_t cover = n > nd ? n : nd;
        k_keys<<<grid_for(cover, 256), 256, 0, s>>>(x, y, z, n, root_half_width, ws.disk_max,
                                                    ws.seg, nd, ws.disk_L, ws.st, kout, vout,
                                                    ws.pack4, m, G);
    } else {
        // few blocks: each ends with one atomic on the same word
        if (!max_ready) k_max_abs<<<grid_for(n, 256, 256), 256, 0, s>>>(x, y, z, n, ws.st);
        k_keys<<<grid_for(n, 256), 256, 0, s>>>(x, y, z, n, root_half_width,
                                                (const unsigned long long *)&ws.st->max_abs,
                                                nullptr, 1, ws.disk_L, ws.st, kout, vout,
                                                ws.pack4, m, G);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// LSD radix sort of (key, index) by 8-bit digits, 8 passes over 63 bits.  Each
// pass: per-tile digit histograms, a per-digit scan over tiles, then a stable
// scatter.  The scatter ranks each wave's 64-item rounds with ballots (wave-private
// running counters), places the tile in LDS in digit order, and then writes it out
// so that each digit's run of the tile leaves as consecutive stores.
constexpr int kSortThreads = 256;
// 2048 items per tile: about two tiles per compute unit at N = 1e6 (4096-item tiles left
// every compute unit with one lone block: 0.225 -> 0.190 ms for the 8 passes)
constexpr int kSortItems = 8;                        // per thread
constexpr int kSortTile = kSortThreads * kSortItems; // 2048
constexpr int kSortWaves = kSortThreads / kWave;

__device__ __forceinline__ uint32_t sort_digit(const uint64_t *keys, const uint32_t *vals,
                                               const uint16_t *dseg, int64_t i, int shift) {
    return dseg ? ((uint32_t)dseg[vals[i]] >> shift) & 255u
                : (uint32_t)(keys[i] >> shift) & 255u;
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_hist(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
             const uint16_t *__restrict__ dseg, int64_t n, int shift, uint32_t *hist,
             int ntiles, const int32_t *__restrict__ skip) {
    __shared__ uint32_t h[256];
    if (skip && *skip) return;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int k = 0; k < kSortItems; k++) {
        const int64_t i = base + k * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[sort_digit(keys, vals, dseg, i, shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: exclusive scan of that digit's tile counts; digit total out.
__global__ void __launch_bounds__(256)
k_radix_scan(uint32_t *hist, int ntiles, uint32_t *totals, const int32_t *__restrict__ skip) {
    __shared__ uint32_t wtot[256 / kWave];
    if (skip && *skip) return;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    uint32_t *row = hist + (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int b0 = 0; b0 < ntiles; b0 += 256) {
        const int i = b0 + threadIdx.x;
        const uint32_t x = i < ntiles ? row[i] : 0u;
        uint32_t v = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(v, o);
            if (lane >= o) v += y;
        }
        if (lane == kWave - 1) wtot[w] = v;
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int k = 0; k < 256 / kWave; k++) {
            if (k < w) before += wtot[k];
            all += wtot[k];
        }
        if (i < ntiles) row[i] = carry + before + v - x;
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__device__ __forceinline__ uint64_t lanemask_lt() {
    uint32_t l = threadIdx.x % kWave;
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// exclusive prefix sum over the block's 256 threads; wsum (4 entries) must not be
// reused by the caller before its next barrier
__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t *wsum) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int k = 0; k < w; k++) add += wsum[k];
    return add + x - v;
}

__global__ void __launch_bounds__(kSortThreads)
k_radix_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                uint64_t *__restrict__ kout, uint32_t *__restrict__ vout,
                const uint16_t *__restrict__ dseg, int64_t n, int shift,
                const uint32_t *__restrict__ hist, const uint32_t *__restrict__ totals,
                int ntiles, const int32_t *__restrict__ skip) {
    __shared__ uint64_t lkey[kSortTile];         // the tile in digit order
    __shared__ uint32_t lval[kSortTile];
    __shared__ uint8_t ldig[kSortTile];
    __shared__ uint32_t wcnt[kSortWaves][256];   // per-wave digit counters
    __shared__ uint32_t lstart[256];             // start of each digit's run in the tile
    __shared__ int32_t delta[256];               // global start minus tile start, per digit
    __shared__ uint32_t wsum_a[kSortWaves], wsum_b[kSortWaves];
    if (skip && *skip) return;
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    for (int k = 0; k < kSortWaves; k++) wcnt[k][t] = 0;
    // global start of digit t's run from this tile: digits below t, then earlier tiles
    const uint32_t gstart = block_excl_scan256(totals[t], wsum_a) +
                            hist[(int64_t)t * ntiles + blockIdx.x];
    // phase 1: this wave's items (a contiguous quarter of the tile), kept in registers
    const int64_t tbase = (int64_t)blockIdx.x * kSortTile;
    const int64_t wbase = tbase + (int64_t)w * (kSortTile / kSortWaves);
    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint32_t dig[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t i = wbase + r * kWave + lane;
        if (i < n) {
            key[r] = kin[i];
            val[r] = vin[i];
            dig[r] = dseg ? ((uint32_t)dseg[val[r]] >> shift) & 255u
                          : (uint32_t)(key[r] >> shift) & 255u;
        } else {
            key[r] = 0;
            val[r] = 0;
            dig[r] = 0;
        }
    }
#pragma unroll
    for (int r = 0; r < kSortItems; r++)
        if (wbase + r * kWave + lane < n) atomicAdd(&wcnt[w][dig[r]], 1u);
    __syncthreads();
    // phase 2: per digit, exclusive prefix over the waves, then over the digits
    uint32_t run = 0;
    for (int k = 0; k < kSortWaves; k++) {
        const uint32_t c = wcnt[k][t];
        wcnt[k][t] = run;
        run += c;
    }
    const uint32_t ls = block_excl_scan256(run, wsum_b);
    lstart[t] = ls;
    delta[t] = (int32_t)(gstart - ls);           // gstart >= ls: see the digit counts
    __syncthreads();
    // phase 3: stable ranks inside each 64-item round, wave-private running counts;
    // items go to their place in the tile's digit order
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const int64_t i = wbase + r * kWave + lane;
        const bool valid = i < n;
        const uint64_t act = __ballot(valid);
        if (act == 0ull) break;
        const uint32_t d = dig[r];
        uint64_t peers = act;
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        if (valid) {
            const uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
            const uint32_t before = wcnt[w][d];
            const uint32_t lpos = lstart[d] + before + rank;
            lkey[lpos] = key[r];
            lval[lpos] = val[r];
            ldig[lpos] = (uint8_t)d;
            const bool leader = (peers & lanemask_lt()) == 0ull;
            __builtin_amdgcn_wave_barrier();
            if (leader) wcnt[w][d] = before + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // phase 4: write the tile out in digit order; a digit's run is contiguous in the
    // output too
    const int cnt = n - tbase < kSortTile ? (int)(n - tbase) : kSortTile;
    for (int j = t; j < cnt; j += kSortThreads) {
        const int64_t pos = (int64_t)delta[ldig[j]] + j;
        if (pos >= 0 && pos < n) {                // always, by the counts; kept as a guard
            kout[pos] = lkey[j];
            vout[pos] = lval[j];
        }
    }
}

hipError_t launch_sort(const Workspace &ws, int64_t n, hipStream_t s) {
    static_assert(kSortTile == kSortTileItems, "tile size of the workspace layout");
    int ntiles = (int)((n + kSortTile - 1) / kSortTile);
    const int npass = 8 + disk_passes(ws.ndisks);
    // launch_keys wrote the keys where an even number of swaps later lands in ws.keys
    uint64_t *ka = ws.keys, *kb = ws.keys_alt;
    uint32_t *va = ws.idx, *vb = ws.idx_alt;
    if (npass % 2 == 1) {
        ka = ws.keys_alt; kb = ws.keys;
        va = ws.idx_alt; vb = ws.idx;
    }
    uint32_t *totals = ws.hist + (int64_t)256 * ntiles;
    for (int pass = 0; pass < npass; pass++) {
        // passes 0-7: key digits; then the disk id, low byte first
        const uint16_t *dseg = pass < 8 ? nullptr : ws.seg;
        const int shift = pass < 8 ? 8 * pass : 8 * (pass - 8);
        k_radix_hist<<<ntiles, kSortThreads, 0, s>>>(ka, va, dseg, n, shift, ws.hist, ntiles,
                                                     nullptr);
        k_radix_scan<<<256, 256, 0, s>>>(ws.hist, ntiles, totals, nullptr);
        k_radix_scatter<<<ntiles, kSortThreads, 0, s>>>(ka, va, kb, vb, dseg, n, shift, ws.hist,
                                                        totals, ntiles, nullptr);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    return hipGetLastError();
}

// Stable sort of (key, value) by the low `bits` bits of the keys, ping-ponging
// between the a and b buffers; returns in *in_b whether the result sits in b.  With
// `skip` given, the passes from `skip_from` on do nothing when *skip is set on the
// device (keys known there to fit the lower digits); an even number of them keeps
// the result where the full sort leaves it.
hipError_t launch_radix_sort(uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb, int64_t n,
                             int bits, uint32_t *hist, bool *in_b, hipStream_t s,
                             const int32_t *skip, int skip_from) {
    const int ntiles = (int)((n + kSortTile - 1) / kSortTile);
    const int npass = (bits + 7) / 8;
    uint32_t *totals = hist + (int64_t)256 * ntiles;
    for (int pass = 0; pass < npass; pass++) {
        const int32_t *sk = skip && pass >= skip_from ? skip : nullptr;
        k_radix_hist<<<ntiles, kSortThreads, 0, s>>>(ka, va, nullptr, n, 8 * pass, hist, ntiles,
                                                     sk);
        k_radix_scan<<<256, 256, 0, s>>>(hist, ntiles, totals, sk);
        k_radix_scatter<<<ntiles, kSortThreads, 0, s>>>(ka, va, kb, vb, nullptr, n, 8 * pass,
                                                        hist, totals, ntiles, sk);
        uint64_t *tk = ka; ka = kb; kb = tk;
        uint32_t *tv = va; va = vb; vb = tv;
    }
    *in_b = npass % 2 == 1;
    return hipGetLastError();
}

// ------------------------------------------------------------------ gathers
// Positions in tree order from the packed records k_keys wrote in input order: one
// 32-byte record per moonlet instead of three scattered 8-byte words (and the scaled
// masses G m from the same record, when k_keys had them: mus != nullptr).
__global__ void k_gather_pack4(const double4 *__restrict__ pack4, const uint32_t *__restrict__ idx,
                              int64_t n, double *__restrict__ xs, double *__restrict__ ys,
                              double *__restrict__ zs, double *__restrict__ mus) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double4 p = pack4[idx[i]];
        xs[i] = p.x;
        ys[i] = p.y;
        zs[i] = p.z;
        if (mus) mus[i] = p.w;
    }
}

__global__ void k_gather1(const double *__restrict__ src, const uint32_t *__restrict__ idx,
                          int64_t n, double *__restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[idx[i]];
}

hipError_t launch_gather_pos(const Workspace &ws, int64_t n, bool with_mus, hipStream_t s) {
    k_gather_pack4<<<grid_for(n, 256), 256, 0, s>>>(ws.pack4, ws.idx, n, ws.xs, ws.ys, ws.zs,
                                                    with_mus ? ws.mus : nullptr);
    return hipGetLastError();
}

__global__ void k_gather_scaled(const double *__restrict__ src, const uint32_t *__restrict__ idx,
                                int64_t n, double scale, double *__restrict__ dst) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = scale * src[idx[i]];
}

hipError_t launch_gather_scaled(const Workspace &ws, const double *src, double scale,
                                double *dst, int64_t n, hipStream_t s) {
    k_gather_scaled<<<grid_for(n, 256), 256, 0, s>>>(src, ws.idx, n, scale, dst);
    return hipGetLastError();
}

// (a, b, c, d)[i] packed into one 32-byte record, in input order (coalesced)
__global__ void k_pack4(const double *__restrict__ a, const double *__restrict__ b,
                        const double *__restrict__ c, const double *__restrict__ d, int64_t n,
                        double4 *__restrict__ out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_double4(a[i], b[i], c[i], d[i]);
}

__global__ void k_gather_vr(const double4 *__restrict__ pack4, const uint32_t *__restrict__ idx,
                            int64_t n, double *__restrict__ as, double *__restrict__ bs,
                            double *__restrict__ cs, double *__restrict__ ds,
                            double4 *__restrict__ vcol) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double4 v = pack4[idx[i]];
        as[i] = v.x;
        bs[i] = v.y;
        cs[i] = v.z;
        ds[i] = v.w;
        vcol[i] = v;
    }
}

// velocities and radii packed in input order (for a gather into tree or mesh order)
hipError_t launch_pack_vr(const Workspace &ws, const double *vx, const double *vy,
                          const double *vz, const double *R, int64_t n, hipStream_t s) {
    k_pack4<<<grid_for(n, 256), 256, 0, s>>>(vx, vy, vz, R, n, ws.pack4);
    return hipGetLastError();
}

// velocities and radii in tree order: packed first (unless `packed`: the kick did it),
// then one record per moonlet instead of four scattered words
hipError_t launch_gather_vr(const Workspace &ws, bool packed, const double *vx,
                            const double *vy, const double *vz, const double *R, int64_t n,
                            hipStream_t s) {
    if (!packed) {
        hipError_t e = launch_pack_vr(ws, vx, vy, vz, R, n, s);
        if (e != hipSuccess) return e;
    }
    k_gather_vr<<<grid_for(n, 256), 256, 0, s>>>(ws.pack4, ws.idx, n, ws.vxs, ws.vys, ws.vzs,
                                                 ws.rads, ws.vcol);
    return hipGetLastError();
}

hipError_t launch_gather(const Workspace &ws, const double *src, double *dst, int64_t n,
                         hipStream_t s) {
    k_gather1<<<grid_for(n, 256), 256, 0, s>>>(src, ws.idx, n, dst);
    return hipGetLastError();
}

}  // namespace ncorp

// Bucket sort of the (Hilbert key, input index) pairs of a plain tree build.
//
// From one step to the next the moonlets move little against the tree, so the order
// of the previous step is nearly the order of this one (Sect. 3.4.6).  The sort uses
// that order for its buckets: the keys the previous build found at ranks
// j kBucketMean (j = 1, 2, ...) split this build's keys into buckets of about
// kBucketMean moonlets each.  Without a previous build (or when the moonlets have
// jumped: a sample of the keys piles up in a few of its buckets) the boundaries come
// from a sorted sample of the keys themselves.  Then
//   count:   the bucket of every pair (binary search over the boundaries) and the
//            moonlets per (bucket, tile);
//   rowscan: per bucket, the exclusive prefix of those counts over the tiles;
//   scatter: every pair to its bucket, stably: a bucket holds its pairs in input
//            order, which is their index order;
//   local:   every bucket sorted by one block with a stable LSD radix sort in LDS
//            over the key bits its keys do not share; the block also records the
//            keys at ranks j kBucketMean for the next build.
// Equal keys thus stay in index order, so the result is the stable sort of the keys,
// and nothing depends on scheduling.  A bucket too large for one LDS batch is sorted
// in batches that are then merged by (key, index) in global memory, so any
// distribution sorts correctly.
#include "ncorp_internal.h"

namespace ncorp {

constexpr int kBsThreads = 256;
constexpr int kBsWaves = kBsThreads / kWave;
constexpr int kBsItems = kBucketTile / kBsThreads;   // rounds per wave, count/scatter
constexpr int kBsLocalThreads = 1024;                 // local sort: one block per bucket
constexpr int kBsLocalWaves = kBsLocalThreads / kWave;
constexpr int kBsRounds = kBucketLDS / kBsLocalThreads;  // rounds per wave, local sort
constexpr int kBsSamplesPer = 4;       // sampled keys per bucket
constexpr int kBsSampleMax = 8192;     // fewer per bucket beyond 2048 buckets
constexpr uint64_t kKeySentinel = ~0ull;  // above every 63-bit key
static_assert(kMaxBuckets <= kBsSampleMax, "at least one sample per bucket");

__device__ __forceinline__ bool pair_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
    return ka < kb || (ka == kb && ia < ib);
}

__device__ __forceinline__ uint64_t bs_lanemask_lt() {
    const uint32_t l = threadIdx.x % kWave;
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// number of boundaries (sk, si)[0..m) that are <= (k, i)
__device__ __forceinline__ int bucket_of(const uint64_t *sk, const uint32_t *si, int m,
                                         uint64_t k, uint32_t i) {
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pair_less(k, i, sk[mid], si[mid])) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int pow2_at_least(int v) {
    int p = 2;
    while (p < v) p <<= 1;
    return p;
}

// Exclusive prefix of v over a block of NT threads, and the block's total.  wsum:
// NT / 64 words of LDS, not reused by the caller before its next barrier.
template <int NT = kBsThreads>
__device__ __forceinline__ uint32_t block_scan(uint32_t v, uint32_t *wsum, uint32_t *total) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < NT / kWave; k++) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    *total = all;
    return before + x - v;
}

// Ascending bitonic sort of (sk, si)[0..P), P a power of two, by a block of NT
// threads (used on the sample only).
template <int NT>
__device__ void bitonic_lds(uint64_t *sk, uint32_t *si, int P) {
    const int half = P >> 1;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < half; t += NT) {
                const int a = 2 * t - (t & (j - 1));
                const int b = a + j;
                const uint64_t ka = sk[a], kb = sk[b];
                const uint32_t ia = si[a], ib = si[b];
                if (pair_less(kb, ib, ka, ia) == ((a & k) == 0)) {
                    sk[a] = kb; si[a] = ib;
                    sk[b] = ka; si[b] = ia;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ boundaries
// One block.  Writes the nb - 1 boundaries: the previous build's when allowed (same n
// and root cube) and a sample of this build's keys spreads over them without piling
// up (no bucket draws more than four times its share of the sample, plus four), else
// those of the sorted sample.  Clears the spill count of this sort.
__global__ void __launch_bounds__(1024)
k_bs_splitters(DevState *st, const uint64_t *__restrict__ keys, const uint32_t *__restrict__ idx,
               int n, int nb, int prev_ok, const SplitKey *__restrict__ prev,
               SplitKey *__restrict__ split) {
    __shared__ uint64_t sk[kBsSampleMax];
    __shared__ uint32_t si[kBsSampleMax];
    __shared__ uint32_t cnt[kMaxBuckets];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) {
        st->bs_spill = 0;
        st->bs_sub_rd = st->bs_sub_wr & 1;
    }
    if (nb <= 1) {
        if (tid == 0) st->bs_prev_used = 0;
        return;
    }
    const int S = nb * kBsSamplesPer < kBsSampleMax ? nb * kBsSamplesPer : kBsSampleMax;
    const bool use_prev = prev_ok && st->bs_valid && st->bs_n == n && st->bs_L == st->L;
    if (use_prev) {
        for (int j = tid; j < nb - 1; j += blockDim.x) {
            sk[j] = prev[j].k;
            si[j] = prev[j].i;
        }
        for (int b = tid; b < nb; b += blockDim.x) cnt[b] = 0;
        if (tid == 0) bad = 0;
        __syncthreads();
        for (int s0 = tid; s0 < S; s0 += 4 * (int)blockDim.x) {
            uint64_t k[4];
            uint32_t x[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int s = s0 + u * (int)blockDim.x;
                if (s < S) {
                    const int p = (int)((int64_t)s * n / S);
                    k[u] = keys[p];
                    x[u] = idx[p];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (s0 + u * (int)blockDim.x < S)
                    atomicAdd(&cnt[bucket_of(sk, si, nb - 1, k[u], x[u])], 1u);
        }
        __syncthreads();
        for (int b = tid; b < nb; b += blockDim.x)
            if (cnt[b] > (uint32_t)((4 * S + 4 * nb) / nb)) bad = 1;
        __syncthreads();
        if (!bad) {
            for (int j = tid; j < nb - 1; j += blockDim.x) split[j] = prev[j];
            if (tid == 0) st->bs_prev_used = 1;
            return;
        }
    }
    // boundaries from a sample at regular positions, sorted
    const int P = pow2_at_least(S);
    for (int s = tid; s < P; s += blockDim.x) {
        if (s < S) {
            const int p = (int)((int64_t)s * n / S);
            sk[s] = keys[p];
            si[s] = idx[p];
        } else {
            sk[s] = kKeySentinel;
            si[s] = ~0u;
        }
    }
    bitonic_lds<1024>(sk, si, P);
    for (int b = 1 + tid; b < nb; b += blockDim.x) {
        const int s = (int)((int64_t)b * S / nb);
        SplitKey v;
        v.k = sk[s];
        v.i = si[s];
        v.pad = 0;
        split[b - 1] = v;
    }
    if (tid == 0) st->bs_prev_used = 0;
}

// ------------------------------------------------------------------ count
// The bucket of every pair (into bkt) and the pairs per bucket of this tile (into
// column `tile` of the bucket-major count matrix).  LDS: boundary keys and indices,
// one counter per bucket.
__global__ void __launch_bounds__(kBsThreads)
k_bs_count(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ idx, int n, int nb,
           int ntiles, const SplitKey *__restrict__ split, uint32_t *__restrict__ bkt,
           uint32_t *__restrict__ cm) {
    extern __shared__ __align__(16) unsigned char smem[];
    uint64_t *sk = reinterpret_cast<uint64_t *>(smem);
    uint32_t *si = reinterpret_cast<uint32_t *>(sk + nb);
    uint32_t *cnt = si + nb;
    const int tid = threadIdx.x;
    for (int j = tid; j < nb - 1; j += kBsThreads) {
        sk[j] = split[j].k;
        si[j] = split[j].i;
    }
    for (int b = tid; b < nb; b += kBsThreads) cnt[b] = 0;
    __syncthreads();
    const int base = blockIdx.x * kBucketTile;
    uint64_t k[kBsItems];
    uint32_t x[kBsItems];
#pragma unroll
    for (int r = 0; r < kBsItems; r++) {
        const int i = base + r * kBsThreads + tid;
        k[r] = 0;
        x[r] = 0;
        if (i < n) {
            k[r] = keys[i];
            x[r] = idx[i];
        }
    }
    // all items' searches advance together: one step per level, count of boundaries
    // <= the pair grown by halving strides
    const int m = nb - 1;
    int lo[kBsItems];
#pragma unroll
    for (int r = 0; r < kBsItems; r++) lo[r] = 0;
    int top = 1;
    while (top * 2 <= m) top *= 2;
    for (int step = m > 0 ? top : 0; step > 0; step >>= 1) {
#pragma unroll
        for (int r = 0; r < kBsItems; r++) {
            const int c = lo[r] + step;
            if (c <= m && !pair_less(k[r], x[r], sk[c - 1], si[c - 1])) lo[r] = c;
        }
    }
#pragma unroll
    for (int r = 0; r < kBsItems; r++) {
        const int i = base + r * kBsThreads + tid;
        if (i < n) {
            bkt[i] = (uint32_t)lo[r];
            atomicAdd(&cnt[lo[r]], 1u);
        }
    }
    __syncthreads();
    for (int b = tid; b < nb; b += kBsThreads) cm[(int64_t)b * ntiles + blockIdx.x] = cnt[b];
}

// ------------------------------------------------------------------ row scan
// One block per bucket: exclusive prefix of its per-tile counts (in place) and its
// total; counts the buckets that need the merging path.
__global__ void __launch_bounds__(kBsThreads)
k_bs_rowscan(DevState *st, uint32_t *__restrict__ cm, int ntiles, uint32_t *__restrict__ total) {
    __shared__ uint32_t wsum[kBsWaves];
    uint32_t *row = cm + (int64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (int t0 = 0; t0 < ntiles; t0 += kBsThreads) {
        const int t = t0 + threadIdx.x;
        const uint32_t c = t < ntiles ? row[t] : 0u;
        uint32_t all;
        const uint32_t ex = block_scan(c, wsum, &all);
        if (t < ntiles) row[t] = carry + ex;
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        total[blockIdx.x] = carry;
        if (carry > (uint32_t)kBucketLDS) atomicAdd(&st->bs_spill, 1);
    }
}

// ------------------------------------------------------------------ scatter
// Every pair to its bucket.  A pair's place: its bucket's start, the pairs of that
// bucket in earlier tiles, in earlier waves of this tile, in earlier rounds of this
// wave, at lower lanes of this round (ballot match over the bucket bits) -- the input
// order.  The tile is first laid out in LDS in bucket order, then written out so that
// each bucket's run of the tile leaves as consecutive stores.  LDS (dynamic): per
// bucket its global start minus its start in the tile, its start in the tile, and
// per-wave counters.  Block 0 also publishes the bucket starts.
struct ScatterLds {
    uint64_t k[kBucketTile];
    uint32_t v[kBucketTile];
    uint16_t b[kBucketTile];
    uint32_t wsum[kBsWaves];
};

__global__ void __launch_bounds__(kBsThreads)
k_bs_scatter(const uint64_t *__restrict__ kin, const uint32_t *__restrict__ vin,
             const uint32_t *__restrict__ bkt, int n, int nb, int ntiles,
             const uint32_t *__restrict__ cm, const uint32_t *__restrict__ total,
             uint32_t *__restrict__ off, uint64_t *__restrict__ kout,
             uint32_t *__restrict__ vout) {
    __shared__ ScatterLds T;
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t *delta = reinterpret_cast<int32_t *>(smem);             // [nb]
    uint32_t *tstart = reinterpret_cast<uint32_t *>(delta + nb);   // [nb]
    uint32_t *wcnt = tstart + nb;                                  // [kBsWaves][nb]
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const int tile = blockIdx.x;
    for (int b = t; b < nb; b += kBsThreads)
#pragma unroll
        for (int k = 0; k < kBsWaves; k++) wcnt[k * nb + b] = 0;
    __syncthreads();
    // this wave's items: a contiguous quarter of the tile
    const int wbase = tile * kBucketTile + w * (kBucketTile / kBsWaves);
    uint64_t key[kBsItems];
    uint32_t val[kBsItems], bk[kBsItems];
#pragma unroll
    for (int r = 0; r < kBsItems; r++) {
        const int i = wbase + r * kWave + lane;
        key[r] = 0;
        val[r] = 0;
        bk[r] = 0;
        if (i < n) {
            key[r] = kin[i];
            val[r] = vin[i];
            bk[r] = bkt[i];
            atomicAdd(&wcnt[w * nb + bk[r]], 1u);
        }
    }
    __syncthreads();
    // per bucket: prefix over the waves, its start in the tile (prefix over the
    // buckets) and in the output (bucket starts, then the tile's prefix)
    uint32_t gcarry = 0, tcarry = 0;
    for (int b0 = 0; b0 < nb; b0 += kBsThreads) {
        const int b = b0 + t;
        uint32_t run = 0;
        if (b < nb)
#pragma unroll
            for (int k = 0; k < kBsWaves; k++) {
                const uint32_t c = wcnt[k * nb + b];
                wcnt[k * nb + b] = run;
                run += c;
            }
        uint32_t tall, gall;
        const uint32_t tex = block_scan(run, T.wsum, &tall);
        __syncthreads();
        const uint32_t g = b < nb ? total[b] : 0u;
        const uint32_t gex = block_scan(g, T.wsum, &gall);
        if (b < nb) {
            const uint32_t gs = gcarry + gex;
            tstart[b] = tcarry + tex;
            delta[b] = (int32_t)(gs + cm[(int64_t)b * ntiles + tile]) - (int32_t)(tcarry + tex);
            if (tile == 0) off[b] = gs;
        }
        gcarry += gall;
        tcarry += tall;
        __syncthreads();
    }
    if (tile == 0 && t == 0) off[nb] = (uint32_t)n;
    const int nbits = nb > 1 ? 32 - __clz(nb - 1) : 0;
    const uint64_t lt = bs_lanemask_lt();
#pragma unroll
    for (int r = 0; r < kBsItems; r++) {
        const int i = wbase + r * kWave + lane;
        const bool valid = i < n;
        const uint64_t act = __ballot(valid);
        if (act == 0ull) continue;
        const uint32_t d = bk[r];
        uint64_t peers = act;
        for (int bit = 0; bit < nbits; bit++) {
            const uint64_t m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        if (valid) {
            const uint64_t lower = peers & lt;
            const uint32_t before = wcnt[w * nb + d];
            const uint32_t lpos = tstart[d] + before + (uint32_t)__popcll(lower);
            T.k[lpos] = key[r];
            T.v[lpos] = val[r];
            T.b[lpos] = (uint16_t)d;
            __builtin_amdgcn_wave_barrier();
            if (lower == 0ull) wcnt[w * nb + d] = before + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const int cnt = n - tile * kBucketTile < kBucketTile ? n - tile * kBucketTile : kBucketTile;
    for (int j = t; j < cnt; j += kBsThreads) {
        const int pos = delta[T.b[j]] + j;
        kout[pos] = T.k[j];
        vout[pos] = T.v[j];
    }
}

// ------------------------------------------------------------------ local sorts
// sub-ranges of the one-pass local sort, and the most pairs it ranks by comparison
// in one sub-range (more: the radix sort)
constexpr int kSubBits = 11;
constexpr int kSubs = 1 << kSubBits;
constexpr int kSubLimit = 64;
constexpr int kAuxWords = 2 * kSubs + 1 > kBsLocalWaves * 256 ? 2 * kSubs + 1 : kBsLocalWaves * 256;
// finer boundaries per bucket (previous order)
constexpr int kSubPer = kBucketMean / kSubStride;
static_assert(kBucketMean % kSubStride == 0 && kSubPer <= 255, "finer boundaries of a bucket");

// LDS of a local sort: the pairs; per-wave digit counters (radix sort) or sub-range
// starts and cursors (one-pass sort); digit starts; reductions
struct LocalLds {
    uint64_t k[kBucketLDS];
    uint32_t v[kBucketLDS];
    uint32_t aux[kAuxWords];
    uint32_t dstart[256];
    uint32_t wsum[kBsLocalWaves];
    uint64_t wmin[kBsLocalWaves], wmax[kBsLocalWaves];
    int crowded;
};

// the fast local sort (previous order): threads per bucket, most pairs per bucket
constexpr int kFastThreads = 256;
constexpr int kFastCap = 2560;
constexpr int kFastRounds = kFastCap / kFastThreads;

// LDS of the fast local sort
struct SubLds {
    uint64_t k[kFastCap];
    uint32_t v[kFastCap];
    uint8_t sb[kFastCap];                    // sub-range of each placed pair
    uint32_t start[kSubPer + 2], cur[kSubPer + 1];
    uint64_t bk[kSubPer];                    // finer boundaries of the bucket
    uint32_t bi[kSubPer];
    uint32_t wsum[kFastThreads / kWave];
    int crowded;
};

// Loads this block's pairs (size <= kBucketLDS, kBsLocalThreads threads, R rounds
// per wave as in radix_sort_local) and the smallest and largest key.
__device__ __forceinline__ void load_local(const uint64_t *kin, const uint32_t *vin, int size,
                                           uint64_t *key, uint32_t *val, bool *valid,
                                           uint64_t &kmin, uint64_t &kmax, LocalLds &L) {
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const int R = (size + kBsLocalThreads - 1) / kBsLocalThreads;
    const int wbase = w * R * kWave;
    kmin = ~0ull;
    kmax = 0;
#pragma unroll
    for (int r = 0; r < kBsRounds; r++) {
        const int p = wbase + r * kWave + lane;
        valid[r] = r < R && p < size;
        key[r] = 0;
        val[r] = 0;
        if (valid[r]) {
            key[r] = kin[p];
            val[r] = vin[p];
            kmin = key[r] < kmin ? key[r] : kmin;
            kmax = key[r] > kmax ? key[r] : kmax;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const uint64_t a = ((uint64_t)__shfl_xor((uint32_t)(kmin >> 32), o) << 32) |
                           __shfl_xor((uint32_t)kmin, o);
        const uint64_t b = ((uint64_t)__shfl_xor((uint32_t)(kmax >> 32), o) << 32) |
                           __shfl_xor((uint32_t)kmax, o);
        kmin = a < kmin ? a : kmin;
        kmax = b > kmax ? b : kmax;
    }
    if (lane == 0) {
        L.wmin[w] = kmin;
        L.wmax[w] = kmax;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBsLocalWaves; k++) {
        kmin = L.wmin[k] < kmin ? L.wmin[k] : kmin;
        kmax = L.wmax[k] > kmax ? L.wmax[k] : kmax;
    }
}

// Local sort on the previous build's order: the keys it had at every kSubStride-th
// rank of this bucket (subs[0..nsub), subs[0] the bucket's own start) split the
// bucket into nsub sub-ranges of about kSubStride pairs; each pair finds its
// sub-range by binary search, sub-ranges get slots (counts, exclusive scan, atomics
// in any order), and a pair's place in its sub-range is the number of pairs of that
// sub-range below it by (key, index).  Writes (kout, vout) and returns true, or
// writes nothing and returns false when some sub-range holds more than kSubLimit
// pairs (moonlets moved far).
__device__ __forceinline__ bool subsplit_sort_local(const uint64_t *kin, const uint32_t *vin,
                                                    int size, const SplitKey *subs, int nsub,
                                                    uint64_t *kout, uint32_t *vout, SubLds &L) {
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const int R = (size + kFastThreads - 1) / kFastThreads;
    const int wbase = w * R * kWave;
    const int m = nsub - 1;                  // inner boundaries subs[1..nsub)
    uint32_t *start = L.start;               // m + 2
    uint32_t *cur = L.cur;                   // m + 1
    for (int q = t; q < m; q += kFastThreads) {
        L.bk[q] = subs[q + 1].k;
        L.bi[q] = subs[q + 1].i;
    }
    for (int q = t; q <= m; q += kFastThreads) start[q] = 0;
    if (t == 0) L.crowded = 0;
    uint64_t key[kFastRounds];
    uint32_t val[kFastRounds];
    bool valid[kFastRounds];
    int sb[kFastRounds];
#pragma unroll
    for (int r = 0; r < kFastRounds; r++) {
        const int p = wbase + r * kWave + lane;
        valid[r] = r < R && p < size;
        key[r] = 0;
        val[r] = 0;
        sb[r] = 0;
        if (valid[r]) {
            key[r] = kin[p];
            val[r] = vin[p];
        }
    }
    __syncthreads();
    int top = 1;
    while (top * 2 <= m) top *= 2;
    for (int step = m > 0 ? top : 0; step > 0; step >>= 1) {
#pragma unroll
        for (int r = 0; r < kFastRounds; r++) {
            const int c = sb[r] + step;
            if (c <= m && !pair_less(key[r], val[r], L.bk[c - 1], L.bi[c - 1])) sb[r] = c;
        }
    }
#pragma unroll
    for (int r = 0; r < kFastRounds; r++)
        if (valid[r]) atomicAdd(&start[sb[r]], 1u);
    __syncthreads();
    const uint32_t c = t <= m ? start[t] : 0u;
    if (c > (uint32_t)kSubLimit) L.crowded = 1;
    uint32_t tot;
    const uint32_t ex = block_scan<kFastThreads>(c, L.wsum, &tot);
    if (t <= m) {
        start[t] = ex;
        cur[t] = ex;
    }
    if (t == 0) start[m + 1] = (uint32_t)size;
    __syncthreads();
    if (L.crowded) return false;
#pragma unroll
    for (int r = 0; r < kFastRounds; r++)
        if (valid[r]) {
            const uint32_t slot = atomicAdd(&cur[sb[r]], 1u);
            L.k[slot] = key[r];
            L.v[slot] = val[r];
            L.sb[slot] = (uint8_t)sb[r];
        }
    __syncthreads();
    for (int j = t; j < size; j += kFastThreads) {
        const uint64_t kj = L.k[j];
        const uint32_t vj = L.v[j];
        const int q = L.sb[j];
        const int s0 = (int)start[q], s1 = (int)start[q + 1];
        int rank = 0;
        for (int u = s0; u < s1; u++) rank += pair_less(L.k[u], L.v[u], kj, vj) ? 1 : 0;
        kout[s0 + rank] = kj;
        vout[s0 + rank] = vj;
    }
    return true;
}

// One-pass local sort: the pairs go to 2^kSubBits sub-ranges by the top bits of
// key - min (counts, exclusive scan, slots claimed by atomics in any order); each
// pair's place in its sub-range is then the number of pairs of that sub-range below
// it by (key, index).  Writes (kout, vout) and returns true, or writes nothing and
// returns false when some sub-range holds more than kSubLimit pairs.
__device__ __forceinline__ bool onepass_sort_local(const uint64_t *kin, const uint32_t *vin,
                                                   int size, uint64_t *kout, uint32_t *vout,
                                                   LocalLds &L) {
    const int t = threadIdx.x;
    uint64_t key[kBsRounds];
    uint32_t val[kBsRounds];
    bool valid[kBsRounds];
    uint64_t kmin, kmax;
    load_local(kin, vin, size, key, val, valid, kmin, kmax, L);
    const uint64_t span = kmax - kmin;
    const int nbits = span ? 64 - __clzll((long long)span) : 0;
    const int sh = nbits > kSubBits ? nbits - kSubBits : 0;
    uint32_t *start = L.aux;                 // kSubs + 1
    uint32_t *cur = L.aux + kSubs + 1;       // kSubs
    for (int i = t; i < kSubs; i += kBsLocalThreads) start[i] = 0;
    if (t == 0) L.crowded = 0;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kBsRounds; r++)
        if (valid[r]) atomicAdd(&start[(uint32_t)((key[r] - kmin) >> sh)], 1u);
    __syncthreads();
    static_assert(kSubs == 2 * kBsLocalThreads, "two sub-ranges per thread");
    const uint32_t c0 = start[2 * t], c1 = start[2 * t + 1];
    if (c0 > (uint32_t)kSubLimit || c1 > (uint32_t)kSubLimit) L.crowded = 1;
    uint32_t tot;
    const uint32_t ex = block_scan<kBsLocalThreads>(c0 + c1, L.wsum, &tot);
    start[2 * t] = ex;
    start[2 * t + 1] = ex + c0;
    cur[2 * t] = ex;
    cur[2 * t + 1] = ex + c0;
    if (t == 0) start[kSubs] = (uint32_t)size;
    __syncthreads();
    if (L.crowded) return false;
#pragma unroll
    for (int r = 0; r < kBsRounds; r++)
        if (valid[r]) {
            const uint32_t slot = atomicAdd(&cur[(uint32_t)((key[r] - kmin) >> sh)], 1u);
            L.k[slot] = key[r];
            L.v[slot] = val[r];
        }
    __syncthreads();
    for (int j = t; j < size; j += kBsLocalThreads) {
        const uint64_t kj = L.k[j];
        const uint32_t vj = L.v[j];
        const uint32_t sb = (uint32_t)((kj - kmin) >> sh);
        const int s0 = (int)start[sb], s1 = (int)start[sb + 1];
        int rank = 0;
        for (int q = s0; q < s1; q++) rank += pair_less(L.k[q], L.v[q], kj, vj) ? 1 : 0;
        kout[s0 + rank] = kj;
        vout[s0 + rank] = vj;
    }
    return true;
}

// lanes of this wave whose 8-bit digit equals d (among the active ones)
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, uint64_t act) {
    uint64_t peers = act;
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
        const uint64_t m = __ballot((d >> bit) & 1u);
        peers &= ((d >> bit) & 1u) ? m : ~m;
    }
    return peers;
}

// Stable LSD radix sort (8-bit digits) of size <= kBucketLDS pairs by key, from
// (kin, vin) to (kout, vout) (may be the same) and to L.k / L.v, by one block of
// kBsLocalThreads.  Only the bits of key - (smallest key) are sorted.  Wave w
// holds positions [w Q, (w + 1) Q), Q = 64 ceil(size / kBsLocalThreads), round r
// lane l at w Q + 64 r + l.  Per pass: the lanes sharing a digit in a round (ballots)
// are counted once by their lowest lane; after the prefix over waves and digits each
// lane's place is its digit's start, the wave's earlier rounds and its rank among
// those lanes.
__device__ __forceinline__ void radix_sort_local(const uint64_t *kin, const uint32_t *vin,
                                                 int size, uint64_t *kout, uint32_t *vout,
                                                 LocalLds &L) {
    const int t = threadIdx.x, w = t / kWave, lane = t % kWave;
    const int R = (size + kBsLocalThreads - 1) / kBsLocalThreads;
    const int wbase = w * R * kWave;
    const uint64_t lt = bs_lanemask_lt();
    uint64_t key[kBsRounds];
    uint32_t val[kBsRounds];
    bool valid[kBsRounds];
    uint64_t kmin, kmax;
    load_local(kin, vin, size, key, val, valid, kmin, kmax, L);
    const uint64_t span = kmax - kmin;
    const int nbits = span ? 64 - __clzll((long long)span) : 0;
    const int passes = (nbits + 7) / 8;
#pragma unroll
    for (int r = 0; r < kBsRounds; r++) key[r] -= kmin;
    for (int pass = 0; pass < passes; pass++) {
        const int shift = 8 * pass;
        if (t < 256)
#pragma unroll
            for (int k = 0; k < kBsLocalWaves; k++) L.aux[k * 256 + t] = 0;
        __syncthreads();
        uint64_t peers[kBsRounds];
#pragma unroll
        for (int r = 0; r < kBsRounds; r++) {
            const uint64_t act = __ballot(valid[r]);
            peers[r] = 0;
            if (act != 0ull) {
                const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
                peers[r] = digit_peers(d, act);
                if (valid[r] && (peers[r] & lt) == 0ull)
                    atomicAdd(&L.aux[w * 256 + d], (uint32_t)__popcll(peers[r]));
            }
        }
        __syncthreads();
        // digit t (threads below 256): exclusive prefix over the waves, then over
        // the digits
        uint32_t run = 0;
        if (t < 256)
#pragma unroll
            for (int k = 0; k < kBsLocalWaves; k++) {
                const uint32_t c = L.aux[k * 256 + t];
                L.aux[k * 256 + t] = run;
                run += c;
            }
        uint32_t tot;
        const uint32_t ds = block_scan<kBsLocalThreads>(run, L.wsum, &tot);
        if (t < 256) L.dstart[t] = ds;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kBsRounds; r++) {
            if (valid[r]) {
                const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
                const uint64_t lower = peers[r] & lt;
                const uint32_t before = L.aux[w * 256 + d];
                const uint32_t pos = L.dstart[d] + before + (uint32_t)__popcll(lower);
                L.k[pos] = key[r];
                L.v[pos] = val[r];
                __builtin_amdgcn_wave_barrier();
                if (lower == 0ull) L.aux[w * 256 + d] = before + (uint32_t)__popcll(peers[r]);
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kBsRounds; r++) {
            const int p = wbase + r * kWave + lane;
            if (valid[r]) {
                key[r] = L.k[p];
                val[r] = L.v[p];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kBsRounds; r++) {
        const int p = wbase + r * kWave + lane;
        if (valid[r]) {
            kout[p] = key[r] + kmin;
            vout[p] = val[r];
            L.k[p] = key[r] + kmin;
            L.v[p] = val[r];
        }
    }
    __syncthreads();
}

// number of pairs in (ka, ia)[lo..hi) that are below (k, i)
__device__ __forceinline__ int count_below(const uint64_t *ka, const uint32_t *ia, int lo, int hi,
                                           uint64_t k, uint32_t i) {
    const int lo0 = lo;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (pair_less(ka[mid], ia[mid], k, i)) lo = mid + 1;
        else hi = mid;
    }
    return lo - lo0;
}

// The next build's boundaries from this sorted bucket [o, o + size): the pairs at
// ranks j kBucketMean (1 <= j < nb) and at ranks k kSubStride.
template <int NT>
__device__ __forceinline__ void write_boundaries(const uint64_t *keys, const uint32_t *idx, int o,
                                                 int size, int nb, SplitKey *next,
                                                 SplitKey *subn) {
    const int tid = threadIdx.x;
    const int j0 = (o + kBucketMean - 1) / kBucketMean > 1 ? (o + kBucketMean - 1) / kBucketMean : 1;
    for (int j = j0 + tid; j < nb && j * kBucketMean < o + size; j += NT) {
        const int p = j * kBucketMean;
        SplitKey v;
        v.k = keys[p];
        v.i = idx[p];
        v.pad = 0;
        next[j - 1] = v;
    }
    const int q0 = (o + kSubStride - 1) / kSubStride;
    for (int q = q0 + tid; q * kSubStride < o + size; q += NT) {
        const int p = q * kSubStride;
        SplitKey v;
        v.k = keys[p];
        v.i = idx[p];
        v.pad = 0;
        subn[q] = v;
    }
}

// Fast local sorts: one block per bucket, for buckets taken from the previous
// order and of at most kFastCap pairs (sub-split sort); a bucket it sorts is marked
// done, with its share of the next build's boundaries written.
__global__ void __launch_bounds__(kFastThreads)
k_bs_fast(const DevState *st, const uint32_t *__restrict__ off, int nb, int n,
          uint64_t *__restrict__ keys, uint32_t *__restrict__ idx, SplitKey *__restrict__ next,
          const SplitKey *sub0, const SplitKey *sub1, SplitKey *nsub0, SplitKey *nsub1,
          uint32_t *__restrict__ done) {
    static_assert(kSubPer < kFastThreads, "one sub-range count per thread");
    __shared__ SubLds L;
    const int b = blockIdx.x;
    const int o = (int)off[b];
    const int size = (int)off[b + 1] - o;
    bool ok = false;
    if (st->bs_prev_used && size > 0 && size <= kFastCap) {
        const SplitKey *subs = st->bs_sub_rd ? sub1 : sub0;
        const int ntot = (n + kSubStride - 1) / kSubStride;
        const int nsub = ntot - b * kSubPer < kSubPer ? ntot - b * kSubPer : kSubPer;
        ok = subsplit_sort_local(keys + o, idx + o, size, subs + (int64_t)b * kSubPer, nsub,
                                 keys + o, idx + o, L);
    }
    if (ok) {
        __threadfence_block();
        __syncthreads();
        write_boundaries<kFastThreads>(keys, idx, o, size, nb, next,
                                       st->bs_sub_rd ? nsub0 : nsub1);
    }
    if (threadIdx.x == 0) done[b] = ok || size <= 0 ? 1u : 0u;
}

// The other buckets, one block each: at most kBucketLDS pairs sorted in LDS (one pass
// over sub-ranges of the key range, or the radix sort where a sub-range is
// crowded); a larger one in kBucketLDS batches (written to the alternate buffers),
// then merged pairwise in global memory until one run remains.  The block also
// stores its share of the next build's boundaries.  LDS: LocalLds (dynamic).
__global__ void __launch_bounds__(kBsLocalThreads)
k_bs_slow(DevState *st, const uint32_t *__restrict__ off, int nb, int n,
          uint64_t *__restrict__ keys, uint32_t *__restrict__ idx, uint64_t *__restrict__ kalt,
          uint32_t *__restrict__ ialt, SplitKey *__restrict__ next, SplitKey *sub0,
          SplitKey *sub1, const uint32_t *__restrict__ done) {
    extern __shared__ __align__(16) unsigned char smem[];
    LocalLds &L = *reinterpret_cast<LocalLds *>(smem);
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const int rd = st->bs_sub_rd;
    SplitKey *subn = rd ? sub0 : sub1;
    if (b == 0 && tid == 0) {
        st->bs_valid = 1;
        st->bs_n = n;
        st->bs_L = st->L;
        st->bs_sub_wr = 1 - rd;
    }
    if (done[b]) return;
    const int o = (int)off[b];
    const int size = (int)off[b + 1] - o;
    if (size <= kBucketLDS) {
        if (!onepass_sort_local(keys + o, idx + o, size, keys + o, idx + o, L))
            radix_sort_local(keys + o, idx + o, size, keys + o, idx + o, L);
        __threadfence_block();
        __syncthreads();
        write_boundaries<kBsLocalThreads>(keys, idx, o, size, nb, next, subn);
        return;
    }
    // batches of kBucketLDS, sorted, into the alternate buffers
    for (int c0 = 0; c0 < size; c0 += kBucketLDS) {
        const int len = size - c0 < kBucketLDS ? size - c0 : kBucketLDS;
        radix_sort_local(keys + o + c0, idx + o + c0, len, kalt + o + c0, ialt + o + c0, L);
    }
    __threadfence_block();
    __syncthreads();
    // pairwise merges: an item's place is its rank in its own run plus the number of
    // items of the other run below it (all pairs are distinct)
    uint64_t *sk_src = kalt, *sk_dst = keys;
    uint32_t *si_src = ialt, *si_dst = idx;
    for (int w = kBucketLDS; w < size; w <<= 1) {          // w: a power of two
        for (int q = tid; q < size; q += kBsLocalThreads) {
            const int s0 = q & ~(2 * w - 1);
            const int a1 = s0 + w < size ? s0 + w : size;
            const int b1 = s0 + 2 * w < size ? s0 + 2 * w : size;
            const uint64_t k = sk_src[o + q];
            const uint32_t i = si_src[o + q];
            int pos;
            if (q < a1) pos = (q - s0) + count_below(sk_src + o, si_src + o, a1, b1, k, i);
            else pos = (q - a1) + count_below(sk_src + o, si_src + o, s0, a1, k, i);
            sk_dst[o + s0 + pos] = k;
            si_dst[o + s0 + pos] = i;
        }
        __threadfence_block();
        __syncthreads();
        uint64_t *tk = sk_src; sk_src = sk_dst; sk_dst = tk;
        uint32_t *ti = si_src; si_src = si_dst; si_dst = ti;
    }
    if (sk_src != keys) {
        for (int q = tid; q < size; q += kBsLocalThreads) {
            keys[o + q] = sk_src[o + q];
            idx[o + q] = si_src[o + q];
        }
        __threadfence_block();
        __syncthreads();
    }
    write_boundaries<kBsLocalThreads>(keys, idx, o, size, nb, next, subn);
}

// ------------------------------------------------------------------ host side
static int64_t n_buckets(int64_t n) { return (n + kBucketMean - 1) / kBucketMean; }

bool bucket_sort_applies(const Workspace &ws, int64_t n) {
    return ws.ndisks <= 1 && n_buckets(n) <= kMaxBuckets && ws.bs_split != nullptr;
}

// launch_keys wrote the pairs to keys_alt / idx_alt; the result lands in keys / idx
hipError_t launch_bucket_sort(const Workspace &ws, int64_t n, hipStream_t s) {
    const int nb = (int)n_buckets(n);
    const int ntiles = (int)((n + kBucketTile - 1) / kBucketTile);
    k_bs_splitters<<<1, 1024, 0, s>>>(ws.st, ws.keys_alt, ws.idx_alt, (int)n, nb,
                                      ws.sort_prev ? 1 : 0, ws.bs_prev, ws.bs_split);
    k_bs_count<<<ntiles, kBsThreads, (size_t)nb * 16, s>>>(ws.keys_alt, ws.idx_alt, (int)n, nb,
                                                           ntiles, ws.bs_split, ws.code, ws.bs_cm);
    k_bs_rowscan<<<nb, kBsThreads, 0, s>>>(ws.st, ws.bs_cm, ntiles, ws.bs_total);
    k_bs_scatter<<<ntiles, kBsThreads, (size_t)nb * 4 * (2 + kBsWaves), s>>>(
        ws.keys_alt, ws.idx_alt, ws.code, (int)n, nb, ntiles, ws.bs_cm, ws.bs_total, ws.bs_off,
        ws.keys, ws.idx);
    k_bs_fast<<<nb, kFastThreads, 0, s>>>(ws.st, ws.bs_off, nb, (int)n, ws.keys, ws.idx,
                                          ws.bs_prev, ws.bs_sub[0], ws.bs_sub[1], ws.bs_sub[0],
                                          ws.bs_sub[1], ws.bs_done);
    k_bs_slow<<<nb, kBsLocalThreads, sizeof(LocalLds), s>>>(ws.st, ws.bs_off, nb, (int)n, ws.keys,
                                                       ws.idx, ws.keys_alt, ws.idx_alt,
                                                       ws.bs_prev, ws.bs_sub[0], ws.bs_sub[1],
                                                       ws.bs_done);
    return hipGetLastError();
}

}  // namespace ncorp

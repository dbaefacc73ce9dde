// Flat octree from Hilbert-sorted keys (Sect. 3.4.1, Sect. 3.4.6).
//
// A cell is a key prefix; it is split iff it holds more than s moonlets and is
// above the depth cap.  With sorted keys the level of each moonlet's leaf follows
// from one sliding window: the level-l cell containing moonlet i holds more than
// s moonlets iff some window [j, j+s] containing i has its two end keys sharing
// l leading digits.  Leaves are then compacted in moonlet order ("entries"), and
// every entry e emits the cells of levels [dv_e, L_e] it starts (dv_e = first
// level where its key differs from the previous moonlet's).  Counting those per
// level gives each cell's breadth-first index directly: cells are ordered by
// level, then by key prefix, so children of consecutive parents are contiguous --
// the ordering the paper's flat tree uses.  No per-level kernel launches.
//
// Batched calls build a forest: moonlets of different disks share no cell (their
// common-prefix length counts as -1), each disk's first moonlet starts all levels
// from 0, so level 0 holds one root per non-empty disk, in disk order.
#include "ncorp_internal.h"

namespace ncorp {

constexpr int kTreeBlock = 1024;
constexpr int kNLev = kMaxDepth + 1;          // levels 0..21

__device__ __forceinline__ int cpl_digits(uint64_t a, uint64_t b) {
    if (a == b) return kMaxDepth;
    return (__clzll((long long)(a ^ b)) - 1) / 3;   // keys use bits 0..62
}

// code: L (bits 0-7), dv (bits 8-15), leaf-start flag (bit 16)
__global__ void __launch_bounds__(kTreeBlock)
k_leaf_levels(const uint64_t *__restrict__ keys, const uint16_t *__restrict__ seg, int64_t n,
              int s, uint32_t *__restrict__ code, int32_t *__restrict__ partials) {
    extern __shared__ uint64_t sk[];                 // keys [b0 - s, b0 + B + s)
    int32_t *sc = (int32_t *)(sk + kTreeBlock + 2 * s);   // c(j), j in [b0 - s, b0 + B)
    uint16_t *sd = (uint16_t *)(sc + kTreeBlock + s);      // disk ids, same span as sk
    __shared__ int32_t red[kTreeBlock / kWave];
    const int64_t b0 = (int64_t)blockIdx.x * kTreeBlock;
    const int span = kTreeBlock + 2 * s;
    for (int k = threadIdx.x; k < span; k += kTreeBlock) {
        int64_t j = b0 - s + k;
        const bool in = j >= 0 && j < n;
        sk[k] = in ? keys[j] : 0ull;
        sd[k] = (in && seg) ? seg[j] : (uint16_t)0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kTreeBlock + s; k += kTreeBlock) {
        int64_t j = b0 - s + k;
        sc[k] = (j >= 0 && j + s < n && sd[k] == sd[k + s]) ? cpl_digits(sk[k], sk[k + s]) : -1;
    }
    __syncthreads();
    const int64_t i = b0 + threadIdx.x;
    int start = 0;
    if (i < n) {
        int M = -1;
        int jlo = (int)(i - s < 0 ? 0 : i - s);
        for (int64_t j = jlo; j <= i; j++) {
            int c = sc[j - (b0 - s)];
            M = c > M ? c : M;
        }
        int L = M + 1 < kMaxDepth ? M + 1 : kMaxDepth;
        int dv;
        if (i == 0 || sd[threadIdx.x + s - 1] != sd[threadIdx.x + s]) dv = 0;
        else {
            uint64_t a = sk[threadIdx.x + s - 1], b = sk[threadIdx.x + s];
            dv = (a == b) ? kMaxDepth + 1 : cpl_digits(a, b) + 1;
        }
        start = dv <= L;
        code[i] = (uint32_t)L | ((uint32_t)dv << 8) | ((uint32_t)start << 16);
    }
    int cnt = __popcll(__ballot(start));
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < kTreeBlock / kWave; k++) t += red[k];
        partials[blockIdx.x] = t;
    }
}

// single block: in-place exclusive scan of up to a few thousand block counts
__global__ void __launch_bounds__(kTreeBlock)
k_scan_small(int32_t *v, int nb, int32_t *total) {
    __shared__ int32_t sh[kTreeBlock];
    int32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kTreeBlock) {
        int i = b0 + threadIdx.x;
        int32_t x = i < nb ? v[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < kTreeBlock; o <<= 1) {
            int32_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) v[i] = carry + sh[threadIdx.x] - x;
        carry += sh[kTreeBlock - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__device__ __forceinline__ uint64_t lanemask_lt64() {
    uint32_t l = threadIdx.x % kWave;
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__global__ void __launch_bounds__(kTreeBlock)
k_emit_entries(const uint32_t *__restrict__ code, int64_t n, const int32_t *__restrict__ partials,
               int32_t *__restrict__ ent_start, uint32_t *__restrict__ ent_code) {
    __shared__ int32_t wsum[kTreeBlock / kWave];
    const int64_t i = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    uint32_t c = i < n ? code[i] : 0u;
    int start = (c >> 16) & 1;
    uint64_t m = __ballot(start);
    int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int before = 0;
    for (int k = 0; k < w; k++) before += wsum[k];
    if (start) {
        int e = partials[blockIdx.x] + before + __popcll(m & lanemask_lt64());
        ent_start[e] = (int32_t)i;
        ent_code[e] = c & 0xffffu;
    }
}

// per block of entries: how many cells each level gets
__global__ void __launch_bounds__(kTreeBlock)
k_level_counts(const uint32_t *__restrict__ ent_code, const int32_t *nleaves_dev,
               int32_t *__restrict__ lcount /* [nb][kNLev] */) {
    __shared__ int32_t acc[kNLev];
    int K = *nleaves_dev;
    if (threadIdx.x < kNLev) acc[threadIdx.x] = 0;
    __syncthreads();
    int64_t e = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    int L = -1, dv = 1;
    if (e < K) {
        uint32_t c = ent_code[e];
        L = c & 255u;
        dv = (c >> 8) & 255u;
    }
    for (int l = 0; l < kNLev; l++) {
        uint64_t m = __ballot(dv <= l && l <= L);
        if (threadIdx.x % kWave == 0 && m) atomicAdd(&acc[l], __popcll(m));
    }
    __syncthreads();
    if (threadIdx.x < kNLev) lcount[(int64_t)blockIdx.x * kNLev + threadIdx.x] = acc[threadIdx.x];
}

// one block per level: exclusive scan over blocks; level totals and offsets
__global__ void __launch_bounds__(256)
k_level_scan(int32_t *lcount, const int32_t *nleaves_dev, DevState *st, int64_t cell_cap) {
    __shared__ int32_t sh[256];
    int K = *nleaves_dev;
    int nb = (K + kTreeBlock - 1) / kTreeBlock;
    int l = blockIdx.x;
    int32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        int b = b0 + threadIdx.x;
        int32_t x = b < nb ? lcount[(int64_t)b * kNLev + l] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {
            int32_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (b < nb) lcount[(int64_t)b * kNLev + l] = carry + sh[threadIdx.x] - x;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) st->level_count[l] = carry;
}


// every entry writes the cells it starts, with parent / first-child links.  Each block
// forms the level offsets from the level totals itself; block 0 also publishes them
// with the cell count and depth (and latches an overflow of cell_cap).
__global__ void __launch_bounds__(kTreeBlock)
k_emit_cells(const int32_t *__restrict__ ent_start, const uint32_t *__restrict__ ent_code,
             const uint64_t *__restrict__ keys, const int32_t *__restrict__ lcount,
             DevState *st, int64_t cell_cap, int32_t *__restrict__ c_level,
             int32_t *__restrict__ c_first, int32_t *__restrict__ c_child,
             int32_t *__restrict__ c_nchild, int32_t *__restrict__ c_parent,
             int32_t *__restrict__ c_entry, uint64_t *__restrict__ c_prefix,
             int32_t *__restrict__ ent_cell, const uint16_t *__restrict__ seg,
             int32_t *__restrict__ disk_root) {
    __shared__ int32_t wcnt[kTreeBlock / kWave][kNLev];
    __shared__ int32_t loff[kNLev];
    const int K = st->nleaves;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (threadIdx.x == 0) {
        int32_t off = 0, maxl = 0;
        for (int l = 0; l < kNLev; l++) {
            loff[l] = off;
            off += st->level_count[l];
            if (st->level_count[l] > 0) maxl = l;
        }
        if (blockIdx.x == 0) {
            for (int l = 0; l < kNLev; l++) st->level_off[l] = loff[l];
            st->level_off[kNLev] = off;
            st->ncells = off;
            st->maxlevel = maxl;
            if (off > cell_cap) {
                atomicOr(&st->status, (int32_t)ST_CAP_CELLS);
                atomicMax((unsigned long long *)&st->required, (unsigned long long)off);
                st->ncells = (int32_t)cell_cap;   // later passes only see what was written
            }
        }
    }
    const int64_t e = (int64_t)blockIdx.x * kTreeBlock + threadIdx.x;
    int L = -1, dv = 1, start = 0;
    uint64_t key = 0;
    if (e < K) {
        uint32_t c = ent_code[e];
        L = c & 255u;
        dv = (c >> 8) & 255u;
        start = ent_start[e];
        key = keys[start];
    }
    // rank of this entry among the level-l cell starts of its wave, for all l
    int32_t rank[kNLev];
    uint64_t lt = lanemask_lt64();
    for (int l = 0; l < kNLev; l++) {
        uint64_t m = __ballot(dv <= l && l <= L);
        rank[l] = __popcll(m & lt);
        if (lane == 0) wcnt[w][l] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < kNLev) {
        int32_t run = 0;
        for (int k = 0; k < kTreeBlock / kWave; k++) {
            int32_t c = wcnt[k][threadIdx.x];
            wcnt[k][threadIdx.x] = run;
            run += c;
        }
    }
    __syncthreads();
    if (e >= K) return;
    const int32_t *lpre = lcount + (int64_t)blockIdx.x * kNLev;
    // exclusive count of level-l cell starts before entry e, all levels
    auto excl = [&](int l) { return lpre[l] + wcnt[w][l] + rank[l]; };
    int lo = dv < 1 ? 0 : dv;           // first level this entry starts
    for (int l = lo; l <= L; l++) {
        int64_t ci = (int64_t)loff[l] + excl(l);
        if (ci >= cell_cap) continue;
        c_level[ci] = l;
        c_first[ci] = start;
        c_entry[ci] = (int32_t)e;
        c_prefix[ci] = key >> (3 * (kMaxDepth - l));
        if (l == 0) disk_root[seg ? seg[start] : 0] = (int32_t)ci;
        if (l < L) {
            c_child[ci] = loff[l + 1] + excl(l + 1);
        } else {
            c_child[ci] = -1;
            c_nchild[ci] = 0;
            ent_cell[e] = (int32_t)ci;
        }
        int32_t par = -1;
        if (l >= 1) {
            if (l - 1 >= dv) par = loff[l - 1] + excl(l - 1);          // also started here
            else par = loff[l - 1] + excl(l - 1) - 1;                  // last start before e
        }
        c_parent[ci] = par;
    }
}

// child counts, moonlet counts and leaf ranges: walk up while this cell (or its
// ancestor) is the last child; the next sibling then starts where it ends.  An
// overflowed tree is unusable: it exposes no cells or leaves to later passes.  Also
// clears the coordinate maximum that the next build's key pass (or a step's drift
// before it) accumulates into, and the first climb's arrival and leaf counters.
__global__ void k_cell_ranges(DevState *st, int64_t n,
                              const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_child,
                              const int32_t *__restrict__ c_parent, const int32_t *__restrict__ c_entry,
                              int32_t *__restrict__ c_count, int32_t *__restrict__ c_nchild,
                              int32_t *__restrict__ c_nent, int32_t *__restrict__ c_arrive,
                              int32_t *__restrict__ climb_next) {
    const bool first = blockIdx.x == 0 && threadIdx.x == 0;
    if (first) st->max_abs = 0.0;
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < kXcds * kCtrStride; t += blockDim.x) climb_next[t] = 0;
    if (st->status & ST_CAP_CELLS) {
        if (first) {
            st->ncells = 0;
            st->nleaves = 0;
        }
        return;
    }
    const int nc = st->ncells, K = st->nleaves;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        c_arrive[c] = 0;
        int par = c_parent[c];
        bool last_child = par >= 0 && (c + 1 >= nc || c_parent[c + 1] != par);
        if (last_child) c_nchild[par] = c - c_child[par] + 1;
        // roots (parent -1) are siblings of each other: the next root starts where
        // a root ends, and the last root ends at n
        int x = c;
        for (int up = 0; up <= kMaxDepth + 1 && x >= 0; up++) {   // bounded by the depth cap
            int px = c_parent[x];
            if (x + 1 < nc && c_parent[x + 1] == px) break;
            x = px;
        }
        int end, eend;
        if (x < 0) { end = (int)n; eend = K; }
        else { end = c_first[x + 1]; eend = c_entry[x + 1]; }
        c_count[c] = end - c_first[c];
        c_nent[c] = eend - c_entry[c];
    }
}


hipError_t launch_build_tree(const Workspace &ws, int64_t n, int s, hipStream_t st) {
    int nb = (int)((n + kTreeBlock - 1) / kTreeBlock);
    size_t shmem = (size_t)(kTreeBlock + 2 * s) * sizeof(uint64_t) +
                   (size_t)(kTreeBlock + s) * sizeof(int32_t) +
                   (size_t)(kTreeBlock + 2 * s) * sizeof(uint16_t);
    const uint16_t *seg = ws.ndisks > 1 ? ws.seg : nullptr;
    k_leaf_levels<<<nb, kTreeBlock, shmem, st>>>(ws.keys, seg, n, s, ws.code, ws.scan_part);
    k_scan_small<<<1, kTreeBlock, 0, st>>>(ws.scan_part, nb, &ws.st->nleaves);
    k_emit_entries<<<nb, kTreeBlock, 0, st>>>(ws.code, n, ws.scan_part, ws.ent_start, ws.ent_code);
    // entries: at most n; launch for the worst case, blocks past K exit
    int32_t *lcount = ws.cnt_a;   // nb x kNLev scratch
    k_level_counts<<<nb, kTreeBlock, 0, st>>>(ws.ent_code, &ws.st->nleaves, lcount);
    k_level_scan<<<kNLev, 256, 0, st>>>(lcount, &ws.st->nleaves, ws.st, ws.cell_cap);
    k_emit_cells<<<nb, kTreeBlock, 0, st>>>(ws.ent_start, ws.ent_code, ws.keys, lcount, ws.st,
                                            ws.cell_cap, ws.c_level, ws.c_first, ws.c_child,
                                            ws.c_nchild, ws.c_parent, ws.c_entry, ws.c_prefix,
                                            ws.ent_cell, seg, ws.disk_root);
    int g = (int)((ws.cell_cap + 255) / 256);
    if (g > 2048) g = 2048;
    k_cell_ranges<<<g, 256, 0, st>>>(ws.st, n, ws.c_first, ws.c_child, ws.c_parent, ws.c_entry,
                                     ws.c_count, ws.c_nchild, ws.c_nent, ws.c_arrive,
                                     ws.climb_next);
    return hipGetLastError();
}

}  // namespace ncorp

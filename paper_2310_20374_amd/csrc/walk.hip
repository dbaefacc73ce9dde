// The falcON dual tree walk (Alg. 2) on the GPU.
//
// The paper's recursion (run iteratively from a stack) becomes one persistent
// launch over a global work queue of cell pairs.  Every wave claims 64 queue
// slots, polls them until their items appear, classifies each pair exactly as
// Alg. 2 does (self pair / brute force before the opening test / well separated /
// brute force after it / split the cell with the larger critical radius) and
// pushes the child pairs with one wave-aggregated atomic.  A single signed counter
// of outstanding items (children added and processed items retired in the same
// atomic) says when the walk is over: at zero no item exists and none can appear.
// A wave that polls for too long without progress latches ST_WALK_STALL and
// leaves, so the kernel always ends.
//
// Pairs classified by the walk do not depend on the order of processing, so the
// lists equal those of the recursive walk; they are then grouped per target and
// sorted, making every later sum independent of the walk's timing.
#include "ncorp_internal.h"

namespace ncorp {

constexpr int kWalkBlock = 256;
constexpr int kWalkGrid = 256;                 // 1024 persistent waves: 4 per CU
constexpr uint64_t kSpinLimit = 1ull << 20;    // empty polls in a row before giving up

__device__ __forceinline__ uint64_t make_item(uint32_t epoch, int a, int b) {
    return ((uint64_t)(epoch & 0xffffu) << 48) | ((uint64_t)(uint32_t)a << 24) | (uint32_t)b;
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int wave_excl_sum(int v, int lane, int &total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(x, o);
        if (lane >= o) x += t;
    }
    total = __shfl(x, kWave - 1);
    return x - v;
}

__global__ void k_walk_init(DevState *st, WalkQueue *wq, uint64_t *queue, uint32_t epoch,
                            int mode) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int nc = st->ncells;
    wq->head = 0;
    wq->epoch = epoch;
    if (mode == 0) { st->nm2l = 0; st->np2p = 0; st->visited = 0; }
    else { st->ncand = 0; }
    if (nc > 0 && !(st->status & kSkipMask)) {
        __hip_atomic_store(&queue[0], make_item(epoch, 0, 0), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        wq->tail = 1;
        wq->outstanding = 1;
    } else {
        wq->tail = 0;
        wq->outstanding = 0;
    }
}

struct WalkArgs {
    DevState *st;
    WalkQueue *wq;
    uint64_t *queue;
    int64_t qcap;
    const WCell *cell;
    int ncs, ncc_pre, ncc_post;
    int2 *m2l, *p2p;                     // outputs (p2p = candidates in collision mode)
    int64_t m2l_cap, p2p_cap;
    int32_t *nm2l, *np2p;
    uint32_t epoch;
};

// Appends the lanes' flagged pairs to a list with one atomic per wave.
__device__ __forceinline__ void emit(bool flag, int a, int b, int lane, int32_t *count,
                                     int2 *list, int64_t cap, DevState *st, int32_t bit) {
    const uint64_t m = __ballot(flag);
    if (!m) return;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    int32_t b0 = 0;
    if (lane == 0) b0 = atomicAdd(count, (int32_t)__popcll(m));
    b0 = __shfl(b0, 0);
    if (flag) {
        const int64_t k = (int64_t)b0 + __popcll(m & lt);
        if (k < cap) list[k] = make_int2(a, b);
    }
    if (lane == 0 && (int64_t)b0 + __popcll(m) > cap) {
        atomicOr(&st->status, bit);
        atomicMax((unsigned long long *)&st->required,
                  (unsigned long long)((int64_t)b0 + __popcll(m)));
    }
}

template <int MODE>
__global__ void __launch_bounds__(kWalkBlock) k_walk(WalkArgs A) {
    const int lane = threadIdx.x % kWave;
    WalkQueue *wq = A.wq;
    const int ncells = A.st->ncells;
    const uint32_t tag = A.epoch & 0xffffu;
    uint64_t spins = 0;
    int64_t visited = 0;
    bool finished = false;
    while (!finished) {
        uint64_t base = 0;
        if (lane == 0) base = atomicAdd((unsigned long long *)&wq->head, (unsigned long long)kWave);
        base = __shfl(base, 0);
        // every later claim lies beyond the queue too: this wave can get no more work
        if (base >= (uint64_t)A.qcap) break;
        const uint64_t slot = base + lane;
        bool pending = slot < (uint64_t)A.qcap;
        while (__any(pending)) {
            uint64_t item = 0;
            if (pending) item = ld_relaxed(&A.queue[slot]);
            const bool valid = pending && (uint32_t)(item >> 48) == tag;
            if (!__any(valid)) {
                // nothing arrived: the walk is over once no pushed item is left
                int64_t o = 0;
                if (lane == 0)
                    o = __hip_atomic_load(&wq->outstanding, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                o = __shfl(o, 0);
                if (o <= 0) { finished = true; break; }
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicOr(&A.st->status, (int32_t)ST_WALK_STALL);
                    finished = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
                continue;
            }
            spins = 0;
            // ---------------- classify the pair (Alg. 2)
            int kind = 0;                       // 0 none, 1 well separated, 2 direct sum
            int npush = 0, split = 0;           // split: 1 self, 2 A, 3 B
            int a = 0, b = 0, na = 0, nb = 0, ca = 0, cb = 0;
            if (valid) {
                a = (int)((item >> 24) & 0xffffffu);
                b = (int)(item & 0xffffffu);
                if (a >= ncells || b >= ncells) {       // cannot happen; never follow it
                    atomicOr(&A.st->status, (int32_t)ST_BAD_ITEM);
                    a = b = 0;
                }
                const WCell wa = A.cell[a];
                na = wa.nchild;
                ca = wa.child;
                if (a == b) {
                    if (wa.count <= A.ncs || na == 0) kind = 2;
                    else { split = 1; npush = na * (na + 1) / 2; }
                } else {
                    const WCell wb = A.cell[b];
                    nb = wb.nchild;
                    cb = wb.child;
                    const int64_t prod = (int64_t)wa.count * (int64_t)wb.count;
                    if (prod < (int64_t)A.ncc_pre) {
                        kind = 2;
                    } else {
                        const double dx = wa.x - wb.x, dy = wa.y - wb.y, dz = wa.z - wb.z;
                        const double d = sqrt(dx * dx + dy * dy + dz * dz);
                        if (wa.rcrit + wb.rcrit <= d) {
                            kind = MODE == 0 ? 1 : 0;          // collisions: nothing
                        } else if (prod < (int64_t)A.ncc_post || (na == 0 && nb == 0)) {
                            kind = 2;
                        } else if (nb == 0 || (na != 0 && wa.rcrit > wb.rcrit)) {
                            split = 2; npush = na;
                        } else {
                            split = 3; npush = nb;
                        }
                    }
                }
            }
            // ---------------- push children (one reservation per wave)
            int tot_push;
            const int off = wave_excl_sum(npush, lane, tot_push);
            int written = 0;
            if (tot_push > 0) {
                uint64_t pbase = 0;
                if (lane == 0)
                    pbase = atomicAdd((unsigned long long *)&wq->tail, (unsigned long long)tot_push);
                pbase = __shfl(pbase, 0);
                const uint64_t my = pbase + (uint64_t)off;
                int j = 0;
                if (split == 1) {
                    for (int x = 0; x < na; x++)
                        for (int y = x; y < na; y++, j++)
                            if (my + j < (uint64_t)A.qcap) {
                                __hip_atomic_store(&A.queue[my + j], make_item(A.epoch, ca + x, ca + y),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                written++;
                            }
                } else if (split == 2) {
                    for (; j < na; j++)
                        if (my + j < (uint64_t)A.qcap) {
                            __hip_atomic_store(&A.queue[my + j], make_item(A.epoch, ca + j, b),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            written++;
                        }
                } else if (split == 3) {
                    for (; j < nb; j++)
                        if (my + j < (uint64_t)A.qcap) {
                            __hip_atomic_store(&A.queue[my + j], make_item(A.epoch, a, cb + j),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            written++;
                        }
                }
                if (pbase + (uint64_t)tot_push > (uint64_t)A.qcap && lane == 0) {
                    atomicOr(&A.st->status, (int32_t)ST_CAP_QUEUE);
                    atomicMax((unsigned long long *)&A.st->required,
                              (unsigned long long)(pbase + tot_push));
                }
            }
            // ---------------- interaction lists
            if (MODE == 0) emit(kind == 1, a, b, lane, A.nm2l, A.m2l, A.m2l_cap, A.st, ST_CAP_M2L);
            emit(kind == 2, a, b, lane, A.np2p, A.p2p, A.p2p_cap, A.st, ST_CAP_P2P);
            // ---------------- retire: children in, processed items out, one atomic
            const int nproc = __popcll(__ballot(valid));
            int wsum = written;
#pragma unroll
            for (int o = kWave / 2; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o);
            if (lane == 0)
                atomicAdd((unsigned long long *)&wq->outstanding,
                          (unsigned long long)(int64_t)(wsum - nproc));
            visited += nproc;
            pending = pending && !valid;
        }
    }
    if (lane == 0 && visited)
        atomicAdd((unsigned long long *)&A.st->visited, (unsigned long long)visited);
}

hipError_t launch_walk(Workspace &ws, int mode, int ncs, int ncc_pre, int ncc_post,
                       hipStream_t s) {
    ws.epoch = (ws.epoch + 1) & 0xffffu;
    if (ws.epoch == 0) {
        // tags wrapped: clear the queue so no stale slot can look valid
        launch_fill_i64((int64_t *)ws.queue, 0, ws.queue_cap, s);
        ws.epoch = 1;
    }
    k_walk_init<<<1, 64, 0, s>>>(ws.st, ws.wq, ws.queue, ws.epoch, mode);
    WalkArgs A;
    A.st = ws.st; A.wq = ws.wq; A.queue = ws.queue; A.qcap = ws.queue_cap;
    A.ncs = ncs; A.ncc_pre = ncc_pre; A.ncc_post = ncc_post;
    A.epoch = ws.epoch;
    if (mode == 0) {
        A.cell = ws.wg;
        A.m2l = ws.m2l; A.m2l_cap = ws.m2l_cap; A.nm2l = &ws.st->nm2l;
        A.p2p = ws.p2p; A.p2p_cap = ws.p2p_cap; A.np2p = &ws.st->np2p;
        k_walk<0><<<kWalkGrid, kWalkBlock, 0, s>>>(A);
    } else {
        A.cell = ws.wc;
        A.m2l = ws.m2l; A.m2l_cap = 0; A.nm2l = &ws.st->nm2l;
        A.p2p = ws.cand; A.p2p_cap = ws.p2p_cap; A.np2p = &ws.st->ncand;
        k_walk<1><<<kWalkGrid, kWalkBlock, 0, s>>>(A);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ lists
// M2L: directed entries grouped by target cell.  P2P: directed entries grouped by
// target leaf -- a pair involving an internal cell A (possible when N_a N_b is
// below a threshold, or N_a <= N_cs) reaches every leaf below A.
__global__ void k_zero_n(int32_t *p, const int32_t *n_dev, int extra) {
    int n = *n_dev + extra;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_count_m2l(const int2 *__restrict__ pairs, const int32_t *npairs_dev,
                            int64_t cap, int32_t *cnt) {
    int np = *npairs_dev;
    if (np > cap) np = (int)cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        int2 q = pairs[i];
        atomicAdd(&cnt[q.x], 1);
        atomicAdd(&cnt[q.y], 1);
    }
}

__global__ void k_fill_m2l(const int2 *__restrict__ pairs, const int32_t *npairs_dev, int64_t cap,
                           const int32_t *__restrict__ off, int32_t *cursor, int32_t *src,
                           int64_t dir_cap) {
    int np = *npairs_dev;
    if (np > cap) np = (int)cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        int2 q = pairs[i];
        int64_t k = (int64_t)off[q.x] + atomicAdd(&cursor[q.x], 1);
        if (k < dir_cap) src[k] = q.y;
        k = (int64_t)off[q.y] + atomicAdd(&cursor[q.y], 1);
        if (k < dir_cap) src[k] = q.x;
    }
}

__global__ void k_count_p2p(const int2 *__restrict__ pairs, const int32_t *npairs_dev, int64_t cap,
                            const int32_t *__restrict__ c_entry, const int32_t *__restrict__ c_nent,
                            int32_t *cnt) {
    int np = *npairs_dev;
    if (np > cap) np = (int)cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        int2 q = pairs[i];
        int e0 = c_entry[q.x], e1 = e0 + c_nent[q.x];
        for (int e = e0; e < e1; e++) atomicAdd(&cnt[e], 1);
        if (q.y != q.x) {
            e0 = c_entry[q.y]; e1 = e0 + c_nent[q.y];
            for (int e = e0; e < e1; e++) atomicAdd(&cnt[e], 1);
        }
    }
}

__global__ void k_fill_p2p(const int2 *__restrict__ pairs, const int32_t *npairs_dev, int64_t cap,
                           const int32_t *__restrict__ c_entry, const int32_t *__restrict__ c_nent,
                           const int32_t *__restrict__ off, int32_t *cursor, int32_t *src,
                           int64_t dir_cap) {
    int np = *npairs_dev;
    if (np > cap) np = (int)cap;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np; i += gridDim.x * blockDim.x) {
        int2 q = pairs[i];
        int e0 = c_entry[q.x], e1 = e0 + c_nent[q.x];
        for (int e = e0; e < e1; e++) {
            int64_t k = (int64_t)off[e] + atomicAdd(&cursor[e], 1);
            if (k < dir_cap) src[k] = q.y;
        }
        if (q.y != q.x) {
            e0 = c_entry[q.y]; e1 = e0 + c_nent[q.y];
            for (int e = e0; e < e1; e++) {
                int64_t k = (int64_t)off[e] + atomicAdd(&cursor[e], 1);
                if (k < dir_cap) src[k] = q.x;
            }
        }
    }
}

// off[n] = total; flags an overflow of the directed list
__global__ void k_set_end(int32_t *off, const int32_t *n_dev, const int32_t *total_dev,
                          int64_t dir_cap, DevState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int32_t t = *total_dev;
    off[*n_dev] = t;
    if ((int64_t)t > dir_cap) {
        atomicOr(&st->status, (int32_t)ST_CAP_LISTS);
        atomicMax((unsigned long long *)&st->required, (unsigned long long)t);
    }
}

// Sort each target's sources ascending: one single-wave block per segment; the
// rank of an element is the number of smaller ones (a segment has no repeats).
__global__ void __launch_bounds__(kWave)
k_sort_segments(const int32_t *n_dev, const int32_t *__restrict__ off, int32_t *src,
                int32_t *tmp, const DevState *st) {
    __shared__ int32_t buf[1024];
    if (st->status & kSkipMask) return;      // lists incomplete
    const int lane = threadIdx.x;
    const int nseg = *n_dev;
    for (int sg = blockIdx.x; sg < nseg; sg += gridDim.x) {
        const int b = off[sg], len = off[sg + 1] - b;
        if (len <= 1) continue;
        if (len <= 1024) {
            for (int i = lane; i < len; i += kWave) buf[i] = src[b + i];
            __syncthreads();
            for (int i = lane; i < len; i += kWave) {
                int v = buf[i], r = 0;
                for (int j = 0; j < len; j++) r += buf[j] < v;
                src[b + r] = v;
            }
            __syncthreads();
        } else {
            for (int i = lane; i < len; i += kWave) tmp[b + i] = src[b + i];
            __syncthreads();
            for (int i = lane; i < len; i += kWave) {
                int v = tmp[b + i], r = 0;
                for (int j = 0; j < len; j++) r += tmp[b + j] < v;
                src[b + r] = v;
            }
            __syncthreads();
        }
    }
}

// directed moonlet interactions of the direct sums: per leaf, its moonlets times
// the moonlets of all its sources, minus the i == j terms
__global__ void k_count_inter(DevState *st, const int32_t *__restrict__ ent_cell,
                              const int32_t *__restrict__ c_count,
                              const int32_t *__restrict__ p2p_off,
                              const int32_t *__restrict__ p2p_src) {
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    unsigned long long tot = 0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K; e += gridDim.x * blockDim.x) {
        const int nt = c_count[ent_cell[e]];
        long long srcs = 0;
        for (int q = p2p_off[e]; q < p2p_off[e + 1]; q++) srcs += c_count[p2p_src[q]];
        tot += (unsigned long long)(nt * srcs - nt);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) tot += __shfl_xor(tot, o);
    if (threadIdx.x % kWave == 0 && tot) atomicAdd((unsigned long long *)&st->p2p_inter, tot);
}

__global__ void k_zero_inter(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->p2p_inter = 0;
}

hipError_t launch_count_interactions(const Workspace &ws, hipStream_t s) {
    k_zero_inter<<<1, 64, 0, s>>>(ws.st);
    k_count_inter<<<256, 256, 0, s>>>(ws.st, ws.ent_cell, ws.c_count, ws.p2p_off, ws.p2p_src);
    return hipGetLastError();
}

static int grid_cap(int64_t n, int block, int cap) {
    int64_t g = (n + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

hipError_t launch_build_lists(const Workspace &ws, int mode, hipStream_t s) {
    if (mode != 0) return hipSuccess;
    DevState *st = ws.st;
    const int gc = grid_cap(ws.cell_cap + 1, 256, 2048);
    const int ge = grid_cap(ws.n_max + 1, 256, 2048);
    // ---- M2L: directed entries by target cell
    k_zero_n<<<gc, 256, 0, s>>>(ws.cnt_a, &st->ncells, 1);
    k_count_m2l<<<1024, 256, 0, s>>>(ws.m2l, &st->nm2l, ws.m2l_cap, ws.cnt_a);
    launch_scan(ws.cnt_a, ws.m2l_off, &st->ncells, ws.cell_cap, ws.scan_part, &st->m2l_dir, s);
    k_set_end<<<1, 64, 0, s>>>(ws.m2l_off, &st->ncells, &st->m2l_dir, ws.m2l_dir_cap, st);
    k_zero_n<<<gc, 256, 0, s>>>(ws.cnt_b, &st->ncells, 1);
    k_fill_m2l<<<1024, 256, 0, s>>>(ws.m2l, &st->nm2l, ws.m2l_cap, ws.m2l_off, ws.cnt_b,
                                    ws.m2l_src, ws.m2l_dir_cap);
    k_sort_segments<<<4096, kWave, 0, s>>>(&st->ncells, ws.m2l_off, ws.m2l_src, ws.cnt_tmp, st);
    // ---- P2P: directed entries by target leaf
    k_zero_n<<<ge, 256, 0, s>>>(ws.cnt_a, &st->nleaves, 1);
    k_count_p2p<<<1024, 256, 0, s>>>(ws.p2p, &st->np2p, ws.p2p_cap, ws.c_entry, ws.c_nent,
                                     ws.cnt_a);
    launch_scan(ws.cnt_a, ws.p2p_off, &st->nleaves, ws.n_max, ws.scan_part, &st->p2p_dir, s);
    k_set_end<<<1, 64, 0, s>>>(ws.p2p_off, &st->nleaves, &st->p2p_dir, ws.p2p_dir_cap, st);
    k_zero_n<<<ge, 256, 0, s>>>(ws.cnt_b, &st->nleaves, 1);
    k_fill_p2p<<<1024, 256, 0, s>>>(ws.p2p, &st->np2p, ws.p2p_cap, ws.c_entry, ws.c_nent,
                                    ws.p2p_off, ws.cnt_b, ws.p2p_src, ws.p2p_dir_cap);
    k_sort_segments<<<4096, kWave, 0, s>>>(&st->nleaves, ws.p2p_off, ws.p2p_src, ws.cnt_tmp, st);
    return hipGetLastError();
}

}  // namespace ncorp

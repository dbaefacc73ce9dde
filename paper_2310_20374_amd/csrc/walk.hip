// The falcON dual tree walk (Alg. 2) on the GPU.
//
// The paper's recursion (run iteratively from a stack) becomes one persistent
// launch over a global work queue of cell pairs.  Every wave claims 128 queue
// slots, polls them until their items appear, classifies each pair exactly as
// Alg. 2 does (self pair / brute force before the opening test / well separated /
// brute force after it / split the cell with the larger critical radius) and
// pushes the child pairs with one wave-aggregated atomic on the tail.  Termination:
// the tail and the count of processed items share one 64-bit word, and a wave
// reserves its items' children and counts those items as processed in the same
// atomic, so processed <= tail at every moment, with equality only when no item
// is waiting or being worked on.  A wave that finds no work reads the word; if
// the two halves are equal the walk is over (the tail can only grow from an item
// not yet counted as processed, and there is none).  A wave that polls for too long without progress latches
// ST_WALK_STALL and leaves, so the kernel always ends.
//
// Pairs classified by the walk do not depend on the order of processing, so the
// lists equal those of the recursive walk.  Besides the plain lists of cell pairs
// the gravity walk appends every pair to per-target lists (each well-separated
// pair to both cells' M2L lists, each direct-sum pair to the direct-sum lists of
// every leaf below either cell).  Their order depends on timing; the consumers
// sort a list before using it, so every sum is independent of the walk's timing.
#include "ncorp_internal.h"
#include "rcrit.h"

namespace ncorp {

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

// Every walk tags its items with a fresh 16-bit tag, advanced on the device, so a
// captured and replayed sequence of walks never meets a stale item carrying its own
// tag.  The init pass derives the walk's tag from the last walk's (which nothing
// writes while it runs) and leaves it in epoch_next, which the walk reads and copies
// to epoch.  When the tag wraps (or the host asks, for a new buffer) the init pass
// clears the queue.
__device__ __forceinline__ uint32_t next_epoch(uint32_t e, bool &wrap) {
    uint32_t n = (e + 1u) & 0xffffu;
    wrap = n == 0u;
    return wrap ? 1u : n;
}

// Resets the queue (one root pair (r, r) per tree of the forest) and, for the
// gravity walk, the per-target list counters; with do_rcrit also the cells' opening
// angles, critical radii and walk records (the gravity climb then leaves them out).
__global__ void k_walk_init(DevState *st, WalkQueue *wq, uint64_t *queue, int64_t qcap,
                            int mode, int32_t *m2l_cnt, int32_t *p2p_cnt, int force_clear,
                            const RcritArgs R, int do_rcrit) {
    const int nc = st->ncells;
    bool wrap = false;
    const uint32_t epoch = next_epoch(wq->epoch, wrap);
    const bool go = nc > 0 && !(st->status & kSkipMask);
    const int nroots = go ? st->level_count[0] : 0;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gstride = (int64_t)gridDim.x * blockDim.x;
    if (do_rcrit && go)
        for (int64_t c = gid; c < nc; c += gstride) rcrit_cell(R, (int)c);
    if (wrap || force_clear)
        for (int64_t i = nroots + gid; i < qcap; i += gstride) queue[i] = 0ull;
    if (mode == 0 && m2l_cnt) {
        const int nl = st->nleaves;
        for (int64_t i = gid; i < nc || i < nl; i += gstride) {
            if (i < nc) m2l_cnt[i] = 0;
            if (i < nl) p2p_cnt[i] = 0;
        }
    }
    for (int64_t r = gid; r < nroots; r += gstride)
        __hip_atomic_store(&queue[r], make_item(epoch, (int)r, (int)r), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (gid != 0) return;
    wq->epoch_next = epoch;
    wq->head = 0;
    if (mode == 0) {
        st->nm2l = 0; st->np2p = 0; st->m2l_slots = 0; st->p2p_slots = 0; st->visited = 0;
        st->nlong_m2l = 0; st->nlong_p2p = 0;
        st->walk_busy_sum = 0; st->walk_busy_max = 0;
    } else {
        st->ncand = 0; st->cand_slots = 0;
    }
    wq->tp = (uint64_t)nroots << 32;
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
    int32_t *nm2l, *np2p;                // exact counts
    int32_t *m2l_slots, *p2p_slots;      // reserved slots
    uint32_t epoch;                      // this walk's tag, read at kernel start
    // gravity: per-target lists
    int32_t *m2l_cnt, *m2l_seg, *p2p_cnt, *p2p_seg;
    int32_t *long_m2l, *long_p2p;        // targets whose list outgrew the LDS sort
    int m2l_stride, p2p_stride;
    int timing;                          // record the waves' busy cycles
};

// Stores v at slot k of target t's list (slot order is arbitrary); k came from
// the target's counter.  The append that makes a list longer than `lds` (what its
// consumer sorts in LDS) records the target in `longs`, for the pre-pass that sorts
// such lists.
__device__ __forceinline__ void store_slot(int k, int32_t *seg, int stride, int t, int v,
                                           int lds, int32_t *nlong, int32_t *longs,
                                           DevState *st) {
    if (k == lds) longs[atomicAdd(nlong, 1)] = t;
    if (k < stride) {
        seg[(int64_t)t * stride + k] = v;
    } else {
        atomicOr(&st->status, (int32_t)ST_CAP_LISTS);
        atomicMax((unsigned long long *)&st->required, (unsigned long long)(k + 1));
    }
}

// A wave's current block of kListChunk slots of a plain cell-pair list.
struct Chunk {
    int64_t base;
    int fill;
    int total;                 // entries this wave emitted (published at exit)
};

// Marks the unused rest of a chunk as gaps (-1, -1).
__device__ __forceinline__ void close_chunk(const Chunk &ch, int lane, int2 *list, int64_t cap) {
    if (ch.base < 0) return;
    for (int i = ch.fill + lane; i < kListChunk; i += kWave)
        if (ch.base + i < cap) list[ch.base + i] = make_int2(-1, -1);
}

// Appends the lanes' flagged pairs to a plain list.  Atomics on one shared
// address are the walk's main cost, so the slot counter is touched once per
// kListChunk entries and the exact count only once per wave, at exit.
__device__ __forceinline__ void emit(bool flag, int a, int b, int lane, Chunk &ch,
                                     int32_t *slots, int2 *list, int64_t cap, DevState *st,
                                     int32_t bit) {
    const uint64_t m = __ballot(flag);
    if (!m) return;
    const int k = __popcll(m);
    if (ch.fill + k > kListChunk) {
        close_chunk(ch, lane, list, cap);
        int32_t nb = 0;
        if (lane == 0) nb = atomicAdd(slots, (int32_t)kListChunk);
        nb = __shfl(nb, 0);
        ch.base = nb;
        ch.fill = 0;
        if (lane == 0 && (int64_t)nb + kListChunk > cap) {
            atomicOr(&st->status, bit);
            atomicMax((unsigned long long *)&st->required,
                      (unsigned long long)((int64_t)nb + kListChunk));
        }
    }
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    if (flag) {
        const int64_t pos = ch.base + ch.fill + __popcll(m & lt);
        if (pos < cap) list[pos] = make_int2(a, b);
    }
    ch.fill += k;
    ch.total += k;
}

// One cell pair, classified as Alg. 2 does.
struct Item {
    int kind;                  // 0 nothing, 1 well separated (M2L), 2 direct sum
    int split;                 // children to push: 1 self pair, 2 split A, 3 split B
    int npush;
    int a, b, na, nb, ca, cb;  // cells, their child counts and first children
    int ea, la, eb, lb;        // first leaf and number of leaves below a and b
};

template <int MODE>
__device__ __forceinline__ Item classify(bool valid, uint64_t item, const WalkArgs &A,
                                         int ncells) {
    Item it = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (!valid) return it;
    int a = (int)((item >> 24) & 0xffffffu);
    int b = (int)(item & 0xffffffu);
    if (a >= ncells || b >= ncells) {                   // cannot happen; never follow it
        atomicOr(&A.st->status, (int32_t)ST_BAD_ITEM);
        a = b = 0;
    }
    it.a = a;
    it.b = b;
    const WCell wa = A.cell[a];
    it.na = wa.nchild;
    it.ca = wa.child;
    it.ea = wa.entry;
    it.la = wa.nent;
    if (a == b) {
        if (wa.count <= A.ncs || it.na == 0) it.kind = 2;
        else { it.split = 1; it.npush = it.na * (it.na + 1) / 2; }
        return it;
    }
    const WCell wb = A.cell[b];
    it.nb = wb.nchild;
    it.cb = wb.child;
    it.eb = wb.entry;
    it.lb = wb.nent;
    const int64_t prod = (int64_t)wa.count * (int64_t)wb.count;
    if (prod < (int64_t)A.ncc_pre) {
        it.kind = 2;
    } else {
        const double dx = wa.x - wb.x, dy = wa.y - wb.y, dz = wa.z - wb.z;
        const double d = sqrt(dx * dx + dy * dy + dz * dz);
        if (wa.rcrit + wb.rcrit <= d) {
            it.kind = MODE == 0 ? 1 : 0;                 // collisions: nothing
        } else if (prod < (int64_t)A.ncc_post || (it.na == 0 && it.nb == 0)) {
            it.kind = 2;
        } else if (it.nb == 0 || (it.na != 0 && wa.rcrit > wb.rcrit)) {
            it.split = 2; it.npush = it.na;
        } else {
            it.split = 3; it.npush = it.nb;
        }
    }
    return it;
}

// Stores an item's child pairs at queue slots my, my+1, ...
__device__ __forceinline__ void push_children(const Item &it, uint64_t my, const WalkArgs &A) {
    int j = 0;
    if (it.split == 1) {
        for (int x = 0; x < it.na; x++)
            for (int y = x; y < it.na; y++, j++)
                if (my + j < (uint64_t)A.qcap)
                    __hip_atomic_store(&A.queue[my + j], make_item(A.epoch, it.ca + x, it.ca + y),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (it.split == 2) {
        for (; j < it.na; j++)
            if (my + j < (uint64_t)A.qcap)
                __hip_atomic_store(&A.queue[my + j], make_item(A.epoch, it.ca + j, it.b),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (it.split == 3) {
        for (; j < it.nb; j++)
            if (my + j < (uint64_t)A.qcap)
                __hip_atomic_store(&A.queue[my + j], make_item(A.epoch, it.a, it.cb + j),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The per-target lists of the gravity walk (see the file header).  A lane's items
// make a stream of appends -- a well-separated pair one to each cell's M2L list, a
// direct-sum pair one to the list of every leaf below either cell -- whose counter
// atomics are issued kAppendBatch at a time, so their latencies overlap.
constexpr int kAppendBatch = 8;

template <int IPL>
__device__ __forceinline__ void append_targets(const Item (&it)[IPL], const WalkArgs &A) {
    int nreq[IPL], ea[IPL], nla[IPL], eb[IPL];
    int total = 0;
#pragma unroll
    for (int k = 0; k < IPL; k++) {
        ea[k] = eb[k] = nla[k] = 0;
        int nlb = 0;
        if (it[k].kind == 2) {
            ea[k] = it[k].ea;
            nla[k] = it[k].la;
            if (it[k].a != it[k].b) {
                eb[k] = it[k].eb;
                nlb = it[k].lb;
            }
        }
        nreq[k] = it[k].kind == 1 ? 2 : (it[k].kind == 2 ? nla[k] + nlb : 0);
        total += nreq[k];
    }
    for (int r0 = 0; r0 < total; r0 += kAppendBatch) {
        int slot[kAppendBatch], tgt[kAppendBatch], val[kAppendBatch];
        bool p2p[kAppendBatch];
#pragma unroll
        for (int q = 0; q < kAppendBatch; q++) {
            int r = r0 + q, k = 0;
#pragma unroll
            for (int m = 0; m + 1 < IPL; m++)
                if (k == m && r >= nreq[m]) { r -= nreq[m]; k = m + 1; }
            int t = 0, v = 0;
            bool isp = false;
#pragma unroll
            for (int m = 0; m < IPL; m++) {
                if (m != k) continue;
                if (it[m].kind == 1) {
                    t = r == 0 ? it[m].a : it[m].b;
                    v = r == 0 ? it[m].b : it[m].a;
                } else {
                    isp = true;
                    t = r < nla[m] ? ea[m] + r : eb[m] + (r - nla[m]);
                    v = r < nla[m] ? it[m].b : it[m].a;
                }
            }
            tgt[q] = t;
            val[q] = v;
            p2p[q] = isp;
            slot[q] = r0 + q < total ? atomicAdd(isp ? &A.p2p_cnt[t] : &A.m2l_cnt[t], 1) : 0;
        }
#pragma unroll
        for (int q = 0; q < kAppendBatch; q++) {
            if (r0 + q >= total) continue;
            if (p2p[q])
                store_slot(slot[q], A.p2p_seg, A.p2p_stride, tgt[q], val[q], kP2PListLDS,
                           &A.st->nlong_p2p, A.long_p2p, A.st);
            else
                store_slot(slot[q], A.m2l_seg, A.m2l_stride, tgt[q], val[q], kM2LListLDS,
                           &A.st->nlong_m2l, A.long_m2l, A.st);
        }
    }
}

// Every wave claims kWave * kItemsPerLane queue slots at a time (lane l takes slots
// l, l + 64, ...), so the shared counters are touched once per that many items.
constexpr int kItemsPerLane = 2;

template <int MODE>
__global__ void __launch_bounds__(kWalkBlock) k_walk(WalkArgs A0) {
    constexpr int IPL = kItemsPerLane;
    WalkArgs A = A0;
    A.epoch = A0.wq->epoch_next;
    if (blockIdx.x == 0 && threadIdx.x == 0) A0.wq->epoch = A.epoch;   // nothing here reads it
    const int lane = threadIdx.x % kWave;
    WalkQueue *wq = A.wq;
    const int ncells = A.st->ncells;
    const uint32_t tag = A.epoch & 0xffffu;
    const long long t_start = (MODE == 0 && A.timing) ? clock64() : 0;
    uint64_t spins = 0;
    int64_t visited = 0;
    bool finished = false;
    Chunk cm = {-1, kListChunk, 0}, cp = {-1, kListChunk, 0};
    while (!finished) {
        uint64_t base = 0;
        if (lane == 0)
            base = atomicAdd((unsigned long long *)&wq->head, (unsigned long long)(kWave * IPL));
        base = __shfl(base, 0);
        // every later claim lies beyond the queue too: this wave can get no more work
        if (base >= (uint64_t)A.qcap) break;
        uint64_t slot[IPL];
        bool pending[IPL];
        bool any_pending = false;
#pragma unroll
        for (int k = 0; k < IPL; k++) {
            slot[k] = base + lane + (uint64_t)k * kWave;
            pending[k] = slot[k] < (uint64_t)A.qcap;
            any_pending = any_pending || pending[k];
        }
        while (__any(any_pending)) {
            bool valid[IPL];
            uint64_t item[IPL];
            bool any_valid = false;
#pragma unroll
            for (int k = 0; k < IPL; k++) {
                item[k] = pending[k] ? ld_relaxed(&A.queue[slot[k]]) : 0;
                valid[k] = pending[k] && (uint32_t)(item[k] >> 48) == tag;
                any_valid = any_valid || valid[k];
            }
            if (!__any(any_valid)) {
                // nothing arrived: the walk is over once every pushed item has
                // been processed (slots beyond the queue were never written).  Idle
                // waves read the shared word only every 8th empty poll and sleep longer
                // the longer they find nothing, so the working waves' atomics on it
                // and their loads meet less traffic.
                int done = 0;
                if ((spins & 7) == 0 && lane == 0) {
                    const uint64_t v = __hip_atomic_load(&wq->tp, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    const uint64_t pr = v & 0xffffffffull;
                    uint64_t t = v >> 32;
                    if (t > (uint64_t)A.qcap) t = (uint64_t)A.qcap;
                    done = pr >= t;
                }
                done = __shfl(done, 0);
                if (done) { finished = true; break; }
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicOr(&A.st->status, (int32_t)ST_WALK_STALL);
                    finished = true;
                    break;
                }
                const int nap = spins < 4 ? 1 : (spins < 16 ? 4 : 16);
                for (int z = 0; z < nap; z++) __builtin_amdgcn_s_sleep(4);
                continue;
            }
            spins = 0;
            Item it[IPL];
            int npush = 0;
#pragma unroll
            for (int k = 0; k < IPL; k++) {
                it[k] = classify<MODE>(valid[k], item[k], A, ncells);
                npush += it[k].npush;
            }
            int nproc = 0;
#pragma unroll
            for (int k = 0; k < IPL; k++) nproc += __popcll(__ballot(valid[k]));
            // ---------------- push children and retire this round's items (one
            // atomic per wave: tail += children, processed += items)
            int tot_push;
            const int off = wave_excl_sum(npush, lane, tot_push);
            if (tot_push > 0) {
                uint64_t pbase = 0;
                if (lane == 0)
                    pbase = atomicAdd((unsigned long long *)&wq->tp,
                                      ((unsigned long long)tot_push << 32) +
                                          (unsigned long long)nproc) >> 32;
                pbase = __shfl(pbase, 0);
                uint64_t my = pbase + (uint64_t)off;
#pragma unroll
                for (int k = 0; k < IPL; k++) {
                    push_children(it[k], my, A);
                    my += (uint64_t)it[k].npush;
                }
                if (pbase + (uint64_t)tot_push > (uint64_t)A.qcap && lane == 0) {
                    atomicOr(&A.st->status, (int32_t)ST_CAP_QUEUE);
                    atomicMax((unsigned long long *)&A.st->required,
                              (unsigned long long)(pbase + tot_push));
                }
            } else if (lane == 0) {
                __hip_atomic_fetch_add(&wq->tp, (uint64_t)nproc, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            // ---------------- interaction lists
#pragma unroll
            for (int k = 0; k < IPL; k++) {
                if (MODE == 0)
                    emit(it[k].kind == 1, it[k].a, it[k].b, lane, cm, A.m2l_slots, A.m2l,
                         A.m2l_cap, A.st, ST_CAP_M2L);
                emit(it[k].kind == 2, it[k].a, it[k].b, lane, cp, A.p2p_slots, A.p2p, A.p2p_cap,
                     A.st, ST_CAP_P2P);
            }
            if (MODE == 0 && A.m2l_cnt) append_targets<IPL>(it, A);
            visited += nproc;
            any_pending = false;
#pragma unroll
            for (int k = 0; k < IPL; k++) {
                pending[k] = pending[k] && !valid[k];
                any_pending = any_pending || pending[k];
            }
        }
    }
    if (MODE == 0) close_chunk(cm, lane, A.m2l, A.m2l_cap);
    close_chunk(cp, lane, A.p2p, A.p2p_cap);
    if (lane == 0) {
        if (MODE == 0 && cm.total) atomicAdd(A.nm2l, cm.total);
        if (cp.total) atomicAdd(A.np2p, cp.total);
    }
    if (lane == 0 && visited)
        atomicAdd((unsigned long long *)&A.st->visited, (unsigned long long)visited);
    if (MODE == 0 && A.timing && lane == 0) {
        const unsigned long long busy = (unsigned long long)(clock64() - t_start);
        atomicAdd((unsigned long long *)&A.st->walk_busy_sum, busy);
        atomicMax((unsigned long long *)&A.st->walk_busy_max, busy);
    }
}

// waves: persistent waves of the gravity walk (the collision walk runs its own count)
hipError_t launch_walk(Workspace &ws, int mode, int ncs, int ncc_pre, int ncc_post, int waves,
                       hipStream_t s, const ncorp_params *rcrit_prm) {
    RcritArgs R = {};
    if (rcrit_prm) R = rcrit_args(ws, *rcrit_prm);
    k_walk_init<<<1024, 256, 0, s>>>(ws.st, ws.wq, ws.queue, ws.queue_cap, mode, ws.m2l_cnt,
                                     ws.p2p_cnt, ws.clear_queue ? 1 : 0, R, rcrit_prm ? 1 : 0);
    ws.clear_queue = false;
    WalkArgs A = {};
    A.st = ws.st; A.wq = ws.wq; A.queue = ws.queue; A.qcap = ws.queue_cap;
    A.ncs = ncs; A.ncc_pre = ncc_pre; A.ncc_post = ncc_post;
    if (mode == 0) {
        A.cell = ws.wg;
        A.m2l = ws.m2l; A.m2l_cap = ws.m2l_cap; A.nm2l = &ws.st->nm2l;
        A.p2p = ws.p2p; A.p2p_cap = ws.p2p_cap; A.np2p = &ws.st->np2p;
        A.m2l_slots = &ws.st->m2l_slots; A.p2p_slots = &ws.st->p2p_slots;
        A.m2l_cnt = ws.m2l_cnt; A.m2l_seg = ws.m2l_seg; A.m2l_stride = ws.m2l_stride;
        A.p2p_cnt = ws.p2p_cnt; A.p2p_seg = ws.p2p_seg; A.p2p_stride = ws.p2p_stride;
        A.long_m2l = ws.long_m2l; A.long_p2p = ws.long_p2p;
        A.timing = ws.timing ? 1 : 0;
        const int grid = (waves > 0 ? waves : kWalkWaves) / (kWalkBlock / kWave);
        k_walk<0><<<grid, kWalkBlock, 0, s>>>(A);
    } else {
        A.cell = ws.wc;
        A.m2l = ws.m2l; A.m2l_cap = 0; A.nm2l = &ws.st->nm2l;
        A.p2p = ws.cand; A.p2p_cap = ws.p2p_cap; A.np2p = &ws.st->ncand;
        A.m2l_slots = &ws.st->m2l_slots; A.p2p_slots = &ws.st->cand_slots;
        k_walk<1><<<kWalkGridCollide, kWalkBlock, 0, s>>>(A);
    }
    return hipGetLastError();
}

// Lists too long for the consumers' LDS sort (the walk recorded their targets)
// are sorted here, in place, one single-wave block per list (rank sort in LDS).
__global__ void __launch_bounds__(kWave)
k_sort_long_lists(const DevState *__restrict__ st, const int32_t *__restrict__ m2l_cnt,
                  int32_t *m2l_seg, int m2l_stride, const int32_t *__restrict__ long_m2l,
                  const int32_t *__restrict__ p2p_cnt, int32_t *p2p_seg, int p2p_stride,
                  const int32_t *__restrict__ long_p2p) {
    extern __shared__ __align__(16) int32_t scr[];   // round_up(largest stride, 4) ints
    if (st->status & kSkipMask) return;
    // the first half of the blocks sorts the M2L lists, the second the direct-sum lists
    const int half = (int)gridDim.x / 2;
    const int which = (int)blockIdx.x < half ? 0 : 1;
    const int32_t *cnt = which == 0 ? m2l_cnt : p2p_cnt;
    int32_t *seg = which == 0 ? m2l_seg : p2p_seg;
    const int stride = which == 0 ? m2l_stride : p2p_stride;
    const int32_t *longs = which == 0 ? long_m2l : long_p2p;
    const int nl = which == 0 ? st->nlong_m2l : st->nlong_p2p;
    const int lane = threadIdx.x;
    for (int q = (int)blockIdx.x - which * half; q < nl; q += half) {
        const int t = longs[q];
        const int len = cnt[t];
        int32_t *list = seg + (int64_t)t * stride;
        const int len4 = (len + 3) & ~3;
        __syncthreads();
        for (int i = lane; i < len4; i += kWave) scr[i] = i < len ? list[i] : 0x7fffffff;
        __syncthreads();
        const int4 *s4 = reinterpret_cast<const int4 *>(scr);
        for (int i = lane; i < len; i += kWave) {
            const int v = scr[i];
            int r = 0;
            #pragma unroll 8
            for (int j = 0; j < len4 / 4; j++) {
                const int4 w = s4[j];
                r += (w.x < v) + (w.y < v) + (w.z < v) + (w.w < v);
            }
            list[r] = v;
        }
    }
}

// directed moonlet interactions of the direct sums: per leaf, its moonlets times
// the moonlets of all its sources, minus the i == j terms
__global__ void k_count_inter(DevState *st, const int32_t *__restrict__ ent_cell,
                              const int32_t *__restrict__ c_count,
                              const int32_t *__restrict__ p2p_cnt,
                              const int32_t *__restrict__ p2p_seg, int stride,
                              const int32_t *__restrict__ m2l_cnt) {
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    unsigned long long tot = 0;
    long long smax = 0;
    int lp = 0, lm = 0;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < K || e < st->ncells;
         e += gridDim.x * blockDim.x) {
        if (e < st->ncells) lm = m2l_cnt[e] > lm ? m2l_cnt[e] : lm;
        if (e >= K) continue;
        lp = p2p_cnt[e] > lp ? p2p_cnt[e] : lp;
        const int nt = c_count[ent_cell[e]];
        const int32_t *seg = p2p_seg + (int64_t)e * stride;
        long long srcs = 0;
        for (int q = 0; q < p2p_cnt[e]; q++) srcs += c_count[seg[q]];
        tot += (unsigned long long)(nt * srcs - nt);
        smax = srcs > smax ? srcs : smax;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o);
        const int a = __shfl_xor(lp, o), b = __shfl_xor(lm, o);
        lp = a > lp ? a : lp;
        lm = b > lm ? b : lm;
        const long long c = __shfl_xor(smax, o);
        smax = c > smax ? c : smax;
    }
    if (threadIdx.x % kWave == 0) {
        if (tot) atomicAdd((unsigned long long *)&st->p2p_inter, tot);
        if (lp) atomicMax(&st->p2p_maxlist, lp);
        if (lm) atomicMax(&st->m2l_maxlist, lm);
        if (smax) atomicMax((unsigned long long *)&st->p2p_src_max, (unsigned long long)smax);
    }
}

__global__ void k_zero_inter(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->p2p_inter = 0;
        st->m2l_maxlist = 0;
        st->p2p_maxlist = 0;
        st->p2p_src_max = 0;
    }
}

hipError_t launch_sort_long_lists(const Workspace &ws, hipStream_t s) {
    if (!ws.m2l_cnt) return hipSuccess;
    const size_t lm = (size_t)((ws.m2l_stride + 3) & ~3) * sizeof(int32_t);
    const size_t lp = (size_t)((ws.p2p_stride + 3) & ~3) * sizeof(int32_t);
    k_sort_long_lists<<<2 * kSortLongBlocks, kWave, lm > lp ? lm : lp, s>>>(
        ws.st, ws.m2l_cnt, ws.m2l_seg, ws.m2l_stride, ws.long_m2l, ws.p2p_cnt, ws.p2p_seg,
        ws.p2p_stride, ws.long_p2p);
    return hipGetLastError();
}

hipError_t launch_count_interactions(const Workspace &ws, hipStream_t s) {
    k_zero_inter<<<1, 64, 0, s>>>(ws.st);
    if (!ws.p2p_cnt) return hipGetLastError();
    k_count_inter<<<256, 256, 0, s>>>(ws.st, ws.ent_cell, ws.c_count, ws.p2p_cnt, ws.p2p_seg,
                                      ws.p2p_stride, ws.m2l_cnt);
    return hipGetLastError();
}

}  // namespace ncorp

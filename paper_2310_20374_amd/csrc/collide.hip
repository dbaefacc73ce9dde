// Collision search on the candidate cell pairs of the collision walk (Alg. 2 with
// "do nothing" for well-separated cells) and the pair test of Sect. 3.1:
//   Delta = (dr.dv)^2 + dv^2 [(R1 + R2)^2 - dr^2]                      (Eq. 1)
//   dt_c  = -(dr.dv + sqrt(Delta)) / dv^2, collision iff 0 <= dt_c <= dt (Eq. 2)
// The arithmetic is FP64 with a fixed operation order and no contraction, and it is
// symmetric under swapping the two moonlets bit for bit (dr and dv only change
// sign), so the pair set is reproducible exactly.
#include "contact.h"

namespace ncorp {

__device__ __forceinline__ int wave_excl_sum_c(int v, int lane, int &total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int t = __shfl_up(x, o);
        if (lane >= o) x += t;
    }
    total = __shfl(x, kWave - 1);
    return x - v;
}

// One wave per candidate cell pair.  B's moonlets are staged in LDS 64 at a time;
// A's moonlets sit on the lanes, and when A has fewer than 64 the lanes split
// B's moonlets into groups.  In a self pair only j > i is tested.
struct PState {
    double x, y, z, vx, vy, vz, R;
    uint32_t id;
};

// Moonlets of cell C (first f, count n) that can reach the sphere (centre s, radius
// rc) of the other cell within the step: |r_a - s| <= R_a + dt |v_a| + rc.  Every
// colliding pair passes (r_crit of a cell bounds R + dt|v| plus the distance of
// each of its moonlets from its centre); the relative margin 1e-9 dwarfs the
// rounding of either side, so no pair the exact test accepts is dropped.  The
// survivors are compacted into out[] in moonlet order; returns their number, or
// -1 if more than `limit` survive.
__device__ __forceinline__ int cull_cell(int f, int n, double4 sph,
                                         const double4 *__restrict__ pcol,
                                         const double *__restrict__ vxs,
                                         const double *__restrict__ vys,
                                         const double *__restrict__ vzs,
                                         const double *__restrict__ rads,
                                         const uint32_t *__restrict__ perm, PState *out,
                                         int limit) {
    const int lane = threadIdx.x;
    int kept = 0;
    for (int c0 = 0; c0 < n; c0 += kWave) {
        bool keep = false;
        PState ps;
        int k = 0;
        if (c0 + lane < n) {
            k = f + c0 + lane;
            // position and R + dt |v|, as the collision climb stored them
            const double4 p = pcol[k];
            ps.x = p.x; ps.y = p.y; ps.z = p.z;
            const double reach = p.w + sph.w;
            const double dx = ps.x - sph.x, dy = ps.y - sph.y, dz = ps.z - sph.z;
            keep = dx * dx + dy * dy + dz * dz <= reach * reach * (1.0 + 1e-9);
        }
        if (keep) {
            ps.vx = vxs[k]; ps.vy = vys[k]; ps.vz = vzs[k]; ps.R = rads[k];
            ps.id = perm[k];
        }
        const uint64_t m = __ballot(keep);
        const int nk = __popcll(m);
        if (kept + nk > limit) return -1;
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        if (keep) out[kept + __popcll(m & lt)] = ps;
        kept += nk;
    }
    return kept;
}

// Every moonlet pair of the candidate cell pair (A, B) (i < j when A == B): lanes
// take moonlets of A, B's moonlets are staged in LDS 64 at a time and split over
// lane groups when A holds fewer than 64.
__device__ __forceinline__ void test_cell_pair(
    int2 pr, PState *sb, const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
    const double *__restrict__ xs, const double *__restrict__ ys, const double *__restrict__ zs,
    const double *__restrict__ vxs, const double *__restrict__ vys,
    const double *__restrict__ vzs, const double *__restrict__ rads,
    const uint32_t *__restrict__ perm, double dt, int64_t *out, int64_t cap, DevState *st,
    unsigned long long &tests) {
    const int lane = threadIdx.x;
    const int fa = c_first[pr.x], na = c_count[pr.x];
    const int fb = c_first[pr.y], nb = c_count[pr.y];
    const bool self = pr.x == pr.y;
    for (int a0 = 0; a0 < na; a0 += 64) {
        const int nac = na - a0 < 64 ? na - a0 : 64;
        int S = 1;
        while (S < nac) S <<= 1;
        const int G = 64 / S, tl = lane % S, grp = lane / S;
        const bool act = tl < nac;
        const int ia = a0 + (act ? tl : 0);
        const int a = fa + ia;
        const double x1 = xs[a], y1 = ys[a], z1 = zs[a], vx1 = vxs[a], vy1 = vys[a],
                     vz1 = vzs[a], R1 = rads[a];
        const uint32_t id1 = perm[a];
        for (int b0 = self ? a0 : 0; b0 < nb; b0 += 64) {
            const int nbc = nb - b0 < 64 ? nb - b0 : 64;
            __syncthreads();
            if (lane < nbc) {
                const int b = fb + b0 + lane;
                PState ps;
                ps.x = xs[b]; ps.y = ys[b]; ps.z = zs[b];
                ps.vx = vxs[b]; ps.vy = vys[b]; ps.vz = vzs[b]; ps.R = rads[b];
                ps.id = perm[b];
                sb[lane] = ps;
            }
            __syncthreads();
            if (!act) continue;
            const int jlo = self ? (ia + 1 - b0 > 0 ? ia + 1 - b0 : 0) : 0;
            // first j >= jlo with j = grp (mod G)
            int j = jlo + ((grp - jlo % G) % G + G) % G;
            for (; j < nbc; j += G) {
                const PState &o = sb[j];
                tests++;
                if (pair_test(x1, y1, z1, vx1, vy1, vz1, R1, o.x, o.y, o.z, o.vx, o.vy, o.vz,
                              o.R, dt))
                    record(out, cap, (unsigned long long *)&st->npairs, id1, o.id);
            }
        }
    }
}

// candidate slots a wave reads at a time; the cell ranges and spheres of both
// sides of all of them are loaded in one go
constexpr int kCandRound = 8;

__global__ void __launch_bounds__(64)
k_collide(DevState *st, const int2 *__restrict__ cand, int64_t cand_cap,
          const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
          const double4 *__restrict__ ccell, const double *__restrict__ xs,
          const double *__restrict__ ys, const double *__restrict__ zs,
          const double *__restrict__ vxs, const double *__restrict__ vys,
          const double *__restrict__ vzs, const double *__restrict__ rads,
          const uint32_t *__restrict__ perm, const double4 *__restrict__ pcol, double dt,
          int64_t *out, int64_t cap, unsigned long long *tests_part) {
    __shared__ PState sp[kWave];    // survivors of both sides (or a staged tile of B)
    if (st->status & kSkipMask) {
        if (threadIdx.x == 0) tests_part[blockIdx.x] = 0;
        return;
    }
    int nc = st->cand_slots;                 // candidate slots, gaps included
    if (nc > cand_cap) nc = (int)cand_cap;
    const int lane = threadIdx.x;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    unsigned long long tests = 0;
    for (int q0 = blockIdx.x * kCandRound; q0 < nc; q0 += gridDim.x * kCandRound) {
        int2 cq = make_int2(-1, -1);
        if (lane < kCandRound && q0 + lane < nc) cq = cand[q0 + lane];
        // lane l < R: side A of candidate l (with B's sphere, for its cull); lane R + l:
        // side B (with A's sphere)
        const int src = lane < kCandRound ? lane : lane - kCandRound;
        const int qa = __shfl(cq.x, src & (kWave - 1)), qb = __shfl(cq.y, src & (kWave - 1));
        const bool side = lane < 2 * kCandRound && qa >= 0;
        const int mine = lane < kCandRound ? qa : qb, other = lane < kCandRound ? qb : qa;
        int cf = 0, cn = 0;
        double4 sph = make_double4(0.0, 0.0, 0.0, 0.0);
        if (side) {
            cf = c_first[mine];
            cn = c_count[mine];
            sph = ccell[other];
        }
        uint64_t live = __ballot(lane < kCandRound && cq.x >= 0);   // gaps are skipped
        while (live) {
            const int l = __ffsll((unsigned long long)live) - 1;
            live &= live - 1;
            const int2 pr = make_int2(__shfl(cq.x, l), __shfl(cq.y, l));
            if (pr.x != pr.y) {
                // distinct cells: keep only moonlets that can reach the other cell
                const int lb = kCandRound + l;
                const int fa = __shfl(cf, l), na = __shfl(cn, l);
                const int fb = __shfl(cf, lb), nb = __shfl(cn, lb);
                int ka = -1, kb = -1;
                __syncthreads();
                if (na + nb <= kWave) {
                    // both sides in one round: lanes [0, na) hold A, [na, na + nb) hold B
                    const bool inA = lane < na, inB = !inA && lane < na + nb;
                    const int sl = inA ? l : lb;
                    const double4 s4 = make_double4(__shfl(sph.x, sl), __shfl(sph.y, sl),
                                                    __shfl(sph.z, sl), __shfl(sph.w, sl));
                    bool keep = false;
                    int k = 0;
                    double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
                    if (inA || inB) {
                        k = inA ? fa + lane : fb + (lane - na);
                        p = pcol[k];
                        const double reach = p.w + s4.w;
                        const double dx = p.x - s4.x, dy = p.y - s4.y, dz = p.z - s4.z;
                        keep = dx * dx + dy * dy + dz * dz <= reach * reach * (1.0 + 1e-9);
                    }
                    const uint64_t mA = __ballot(keep && inA), mB = __ballot(keep && inB);
                    ka = __popcll(mA);
                    kb = __popcll(mB);
                    if (keep) {
                        PState ps;
                        ps.x = p.x; ps.y = p.y; ps.z = p.z;
                        ps.vx = vxs[k]; ps.vy = vys[k]; ps.vz = vzs[k]; ps.R = rads[k];
                        ps.id = perm[k];
                        sp[inA ? __popcll(mA & lt) : ka + __popcll(mB & lt)] = ps;
                    }
                } else {
                    const double4 sA = make_double4(__shfl(sph.x, l), __shfl(sph.y, l),
                                                    __shfl(sph.z, l), __shfl(sph.w, l));
                    const double4 sB = make_double4(__shfl(sph.x, lb), __shfl(sph.y, lb),
                                                    __shfl(sph.z, lb), __shfl(sph.w, lb));
                    ka = cull_cell(fa, na, sA, pcol, vxs, vys, vzs, rads, perm, sp, kWave);
                    kb = ka < 0 ? -1
                                : cull_cell(fb, nb, sB, pcol, vxs, vys, vzs, rads, perm, sp + ka,
                                            kWave - ka);
                }
                __syncthreads();
                if (ka >= 0 && kb >= 0) {
                    const int tot = ka * kb;
                    for (int t = lane; t < tot; t += kWave) {
                        const PState &p = sp[t / kb], &o = sp[ka + t % kb];
                        tests++;
                        if (pair_test(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.R, o.x, o.y, o.z, o.vx,
                                      o.vy, o.vz, o.R, dt))
                            record(out, cap, (unsigned long long *)&st->npairs, p.id, o.id);
                    }
                    continue;
                }
            }
            test_cell_pair(pr, sp, c_first, c_count, xs, ys, zs, vxs, vys, vzs, rads, perm, dt,
                           out, cap, st, tests);
        }
    }
    // per-block partials, summed by k_sum_u64: one atomic per wave on a single
    // counter would serialise all blocks of the grid
    for (int o = 32; o > 0; o >>= 1) tests += __shfl_xor(tests, o);
    if (lane == 0) tests_part[blockIdx.x] = tests;
}

// dst (+)= the sum of n partials, in a fixed order
__global__ void __launch_bounds__(1024)
k_sum_u64(const unsigned long long *__restrict__ part, int64_t n, unsigned long long *dst,
          int add) {
    __shared__ unsigned long long red[1024 / kWave];
    unsigned long long v = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) v += part[i];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < 1024 / kWave; k++) t += red[k];
        *dst = add ? *dst + t : t;
    }
}

hipError_t launch_sum_u64(const unsigned long long *part, int64_t n, unsigned long long *dst,
                          bool add, hipStream_t s) {
    k_sum_u64<<<1, 1024, 0, s>>>(part, n, dst, add ? 1 : 0);
    return hipGetLastError();
}

__global__ void k_collide_init(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { st->npairs = 0; st->col_tests = 0; }
}

hipError_t launch_collide_reset(const Workspace &ws, hipStream_t s) {
    k_collide_init<<<1, 64, 0, s>>>(ws.st);
    return hipGetLastError();
}

// rank sort of the (distinct) pair keys: rank = number of smaller keys
__global__ void __launch_bounds__(256)
k_rank_pairs(const DevState *__restrict__ st, const int64_t *__restrict__ in, int64_t cap,
             int64_t *__restrict__ out) {
    __shared__ int64_t tile[1024];
    int64_t n = st->npairs;
    if (n > cap) n = cap;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < n; base += (int64_t)gridDim.x * 256) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < n ? in[i] : 0;
        int64_t r = 0;
        for (int64_t t0 = 0; t0 < n; t0 += 1024) {
            __syncthreads();
            for (int k = threadIdx.x; k < 1024; k += 256)
                tile[k] = t0 + k < n ? in[t0 + k] : INT64_MAX;
            __syncthreads();
            const int lim = n - t0 < 1024 ? (int)(n - t0) : 1024;
            for (int k = 0; k < lim; k++) r += tile[k] < v;
        }
        if (i < n) out[r] = v;
    }
}

__global__ void k_emit_pairs(const DevState *__restrict__ st, const int64_t *__restrict__ sorted,
                             int64_t tmp_cap, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev,
                             int triple, int step, int64_t *cursor) {
    int64_t n = st->npairs;
    int64_t m = n < tmp_cap ? n : tmp_cap;
    int64_t base = triple ? *cursor : 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = sorted[k];
        const int64_t o = base + k;
        if (o >= cap) continue;
        if (triple) {
            pairs[3 * o] = step;
            pairs[3 * o + 1] = v >> 32;
            pairs[3 * o + 2] = v & 0xffffffffll;
        } else {
            pairs[2 * o] = v >> 32;
            pairs[2 * o + 1] = v & 0xffffffffll;
        }
    }
}

__global__ void k_pairs_done(DevState *st, int64_t *n_pairs_dev, int64_t cap, int64_t tmp_cap,
                             int triple, int64_t *cursor) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t n = st->npairs;
    *n_pairs_dev = n;
    int64_t base = triple ? *cursor : 0;
    if (n > tmp_cap || base + n > cap) {
        atomicOr(&st->status, (int32_t)ST_CAP_PAIRS);
        atomicMax((unsigned long long *)&st->required, (unsigned long long)(base + n));
    }
    if (triple) *cursor = base + n;
}

// ---------------------------------------------------------------- candidates
// Collision candidates from the gravity walk of the same tree.  That walk splits
// the set of all moonlet pairs into its interactions exactly once each (well-
// separated cell pairs, direct-sum cell pairs, direct-sum self cells).  A moonlet
// pair of an interaction (A, B) can collide only if the collision spheres of the
// two leaves holding them overlap (Eqs. 8-9 bound every moonlet's reach by its
// leaf's r_crit), and, for a well-separated pair, only if the spheres of A and B
// themselves overlap.  So the leaf pairs of all interactions whose spheres overlap
// (and every leaf with two moonlets or more, with itself) are candidates covering
// every colliding pair exactly once: the pair set is the collision walk's.  The
// spheres are compared with a relative margin of 1e-9, far above rounding.
__device__ __forceinline__ bool spheres_meet(const double4 &a, const double4 &b) {
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const double rs = (a.w + b.w) * (1.0 + 1e-9);
    return dx * dx + dy * dy + dz * dz < rs * rs;
}

// Counts (out == nullptr) or writes the candidate leaf pairs of one interaction.
__device__ __forceinline__ int leaf_candidates(int2 pr, bool separated,
                                               const double4 *__restrict__ ccell,
                                               const int32_t *__restrict__ c_entry,
                                               const int32_t *__restrict__ c_nent,
                                               const int32_t *__restrict__ c_count,
                                               const int32_t *__restrict__ ent_cell, int2 *out,
                                               int64_t pos, int64_t cap) {
    if (pr.x < 0) return 0;
    if (separated && !spheres_meet(ccell[pr.x], ccell[pr.y])) return 0;
    const bool self = pr.x == pr.y;
    const int ea = c_entry[pr.x], na = c_nent[pr.x];
    const int eb = c_entry[pr.y], nb = c_nent[pr.y];
    int k = 0;
    for (int i = 0; i < na; i++) {
        const int la = ent_cell[ea + i];
        const double4 sa = ccell[la];
        // four leaves of B at a time: their loads are independent of each other
        for (int j0 = self ? i : 0; j0 < nb; j0 += 4) {
            int lb[4];
            double4 sb[4];
#pragma unroll
            for (int u = 0; u < 4; u++) lb[u] = j0 + u < nb ? ent_cell[eb + j0 + u] : la;
#pragma unroll
            for (int u = 0; u < 4; u++) sb[u] = ccell[lb[u]];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (j0 + u >= nb) continue;
                const bool take = la == lb[u] ? c_count[la] > 1 : spheres_meet(sa, sb[u]);
                if (!take) continue;
                if (out && pos + k < cap) out[pos + k] = make_int2(la, lb[u]);
                k++;
            }
        }
    }
    return k;
}

constexpr int kCandBlock = 256;
constexpr int kCandGrid = 8192;

// The candidates are counted per block, the block counts scanned, and the blocks
// write their candidates at their offsets: no contended atomics, no gaps.  Block b
// takes list slots (r * grid + b) * kCandBlock + t, r = 0, 1, ... in both passes.
struct CandLists {
    const int2 *m2l, *p2p;
    int64_t nm, total;
};

__device__ __forceinline__ CandLists cand_lists(const DevState *st, const int2 *m2l,
                                                int64_t m2l_cap, const int2 *p2p,
                                                int64_t p2p_cap) {
    CandLists L;
    L.m2l = m2l;
    L.p2p = p2p;
    L.nm = st->m2l_slots < m2l_cap ? st->m2l_slots : m2l_cap;
    const int64_t np = st->p2p_slots < p2p_cap ? st->p2p_slots : p2p_cap;
    L.total = L.nm + np;
    return L;
}

// block-wide exclusive prefix of v (kCandBlock threads); returns the block total
__device__ __forceinline__ int block_excl(int v, int &excl, int *wtot) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int tot;
    const int off = wave_excl_sum_c(v, lane, tot);
    if (lane == 0) wtot[w] = tot;
    __syncthreads();
    int before = 0, all = 0;
    for (int k = 0; k < kCandBlock / kWave; k++) {
        if (k < w) before += wtot[k];
        all += wtot[k];
    }
    __syncthreads();
    excl = before + off;
    return all;
}

__global__ void __launch_bounds__(kCandBlock)
k_cand_count(const DevState *__restrict__ st, const int2 *__restrict__ m2l, int64_t m2l_cap,
             const int2 *__restrict__ p2p, int64_t p2p_cap, const double4 *__restrict__ ccell,
             const int32_t *__restrict__ c_entry, const int32_t *__restrict__ c_nent,
             const int32_t *__restrict__ c_count, const int32_t *__restrict__ ent_cell,
             int32_t *__restrict__ blk) {
    __shared__ int wtot[kCandBlock / kWave];
    const CandLists L = cand_lists(st, m2l, m2l_cap, p2p, p2p_cap);
    const bool skip = (st->status & kSkipMask) != 0;
    int sum = 0;
    for (int64_t q0 = (int64_t)blockIdx.x * kCandBlock; q0 < L.total && !skip;
         q0 += (int64_t)gridDim.x * kCandBlock) {
        const int64_t q = q0 + threadIdx.x;
        int2 pr = make_int2(-1, -1);
        const bool sep = q < L.nm;
        if (q < L.total) pr = sep ? L.m2l[q] : L.p2p[q - L.nm];        // gaps are (-1, -1)
        const int cnt = leaf_candidates(pr, sep, ccell, c_entry, c_nent, c_count, ent_cell,
                                        nullptr, 0, 0);
        int excl;
        sum += block_excl(cnt, excl, wtot);
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = sum;
}

// exclusive scan of the block counts (one block); the total is the candidate count
__global__ void __launch_bounds__(1024) k_cand_scan(DevState *st, int32_t *blk, int nb) {
    __shared__ int32_t wtot[1024 / kWave];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024) {
        const int i = b0 + threadIdx.x;
        const int32_t x = i < nb ? blk[i] : 0;
        int32_t v = x;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int32_t y = __shfl_up(v, o);
            if (lane >= o) v += y;
        }
        if (lane == kWave - 1) wtot[w] = v;
        __syncthreads();
        int32_t before = 0, all = 0;
        for (int k = 0; k < 1024 / kWave; k++) {
            if (k < w) before += wtot[k];
            all += wtot[k];
        }
        if (i < nb) blk[i] = carry + before + v - x;
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        st->ncand = carry;
        st->cand_slots = carry;
    }
}

__global__ void __launch_bounds__(kCandBlock)
k_cand_write(DevState *st, const int2 *__restrict__ m2l, int64_t m2l_cap,
             const int2 *__restrict__ p2p, int64_t p2p_cap, const double4 *__restrict__ ccell,
             const int32_t *__restrict__ c_entry, const int32_t *__restrict__ c_nent,
             const int32_t *__restrict__ c_count, const int32_t *__restrict__ ent_cell,
             const int32_t *__restrict__ blk, int2 *cand, int64_t cand_cap) {
    __shared__ int wtot[kCandBlock / kWave];
    if (st->status & kSkipMask) return;
    const CandLists L = cand_lists(st, m2l, m2l_cap, p2p, p2p_cap);
    int64_t run = blk[blockIdx.x];
    for (int64_t q0 = (int64_t)blockIdx.x * kCandBlock; q0 < L.total;
         q0 += (int64_t)gridDim.x * kCandBlock) {
        const int64_t q = q0 + threadIdx.x;
        int2 pr = make_int2(-1, -1);
        const bool sep = q < L.nm;
        if (q < L.total) pr = sep ? L.m2l[q] : L.p2p[q - L.nm];
        const int cnt = leaf_candidates(pr, sep, ccell, c_entry, c_nent, c_count, ent_cell,
                                        nullptr, 0, 0);
        int excl;
        const int all = block_excl(cnt, excl, wtot);
        const int64_t pos = run + excl;
        if (cnt) leaf_candidates(pr, sep, ccell, c_entry, c_nent, c_count, ent_cell, cand, pos,
                                 cand_cap);
        if (cnt && pos + cnt > cand_cap) {
            atomicOr(&st->status, (int32_t)ST_CAP_P2P);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)(pos + cnt));
        }
        run += all;
    }
}

hipError_t launch_candidates_from_lists(const Workspace &ws, hipStream_t s) {
    // one pass of blocks over the list slots when the lists are short enough
    int64_t g = (ws.m2l_cap + ws.p2p_cap + kCandBlock - 1) / kCandBlock;
    if (g > kCandGrid) g = kCandGrid;
    if (g < 1) g = 1;
    k_cand_count<<<(int)g, kCandBlock, 0, s>>>(ws.st, ws.m2l, ws.m2l_cap, ws.p2p, ws.p2p_cap,
                                               ws.ccell, ws.c_entry, ws.c_nent, ws.c_count,
                                               ws.ent_cell, ws.cand_blk);
    k_cand_scan<<<1, 1024, 0, s>>>(ws.st, ws.cand_blk, (int)g);
    k_cand_write<<<(int)g, kCandBlock, 0, s>>>(ws.st, ws.m2l, ws.m2l_cap, ws.p2p, ws.p2p_cap,
                                               ws.ccell, ws.c_entry, ws.c_nent, ws.c_count,
                                               ws.ent_cell, ws.cand_blk, ws.cand, ws.p2p_cap);
    return hipGetLastError();
}

// ---------------------------------------------------------------- resolution
// Hard-sphere resolution of the pairs found (Sect. 5.1-5.2), one block.  Pairs are
// taken in increasing (dt_c, i, j) and a moonlet collides at most once per step:
// this greedy matching is reached in rounds, each accepting every live pair that
// is the earliest live pair of both its moonlets (the earliest live pair of all is
// always one, so every round makes progress) and dropping the live pairs that
// touch a moonlet just matched -- the same set as taking the pairs one by one.
// The pair list is sorted by (i, j), so its index breaks ties of dt_c.
__device__ __forceinline__ bool earlier(const double *dtc, int p, int q) {
    return dtc[p] < dtc[q] || (dtc[p] == dtc[q] && p < q);
}

__device__ __forceinline__ void keep_earliest(int32_t *slot, int p, const double *dtc) {
    int cur = *slot;
    while (cur < 0 || earlier(dtc, p, cur)) {
        const int old = atomicCAS(slot, cur, p);
        if (old == cur) break;
        cur = old;
    }
}

constexpr int kResolveThreads = 1024;

__global__ void __launch_bounds__(kResolveThreads)
k_resolve(DevState *st, const int64_t *__restrict__ keys, int64_t pair_cap, double *x,
          double *y, double *z, double *vx, double *vy, double *vz,
          const double *__restrict__ m, const double *__restrict__ R, double dt, double f,
          double *dtc, int32_t *flag, int32_t *mbest, int32_t *mmatch, int64_t *pairs,
          int64_t cap, int64_t *n_pairs_dev, int step, int64_t *cursor) {
    __shared__ int wsum[kResolveThreads / kWave];
    __shared__ int64_t s_run, s_base;
    const int tid = threadIdx.x, lane = tid % kWave, w = tid / kWave;
    const int T = blockDim.x;
    int64_t np = st->npairs;
    if (np > pair_cap) {                  // the list is incomplete: resolve nothing
        if (tid == 0) {
            atomicOr(&st->status, (int32_t)ST_CAP_PAIRS);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)np);
        }
        np = 0;
    }
    if (st->status & kSkipMask) np = 0;
    // flag: 0 dropped, 1 live, 2 resolved
    for (int64_t p = tid; p < np; p += T) {
        const int i = (int)(keys[p] >> 32), j = (int)(keys[p] & 0xffffffffll);
        const double t = contact_time(x[i], y[i], z[i], vx[i], vy[i], vz[i], R[i], x[j], y[j],
                                      z[j], vx[j], vy[j], vz[j], R[j], dt);
        dtc[p] = t;
        flag[p] = t >= 0.0 ? 1 : 0;
        mmatch[i] = 0;
        mmatch[j] = 0;
    }
    __syncthreads();
    for (int64_t round = 0; round <= np; round++) {
        for (int64_t p = tid; p < np; p += T)
            if (flag[p] == 1) {
                mbest[(int)(keys[p] >> 32)] = -1;
                mbest[(int)(keys[p] & 0xffffffffll)] = -1;
            }
        __syncthreads();
        for (int64_t p = tid; p < np; p += T)
            if (flag[p] == 1) {
                keep_earliest(&mbest[(int)(keys[p] >> 32)], (int)p, dtc);
                keep_earliest(&mbest[(int)(keys[p] & 0xffffffffll)], (int)p, dtc);
            }
        __syncthreads();
        for (int64_t p = tid; p < np; p += T)
            if (flag[p] == 1) {
                const int i = (int)(keys[p] >> 32), j = (int)(keys[p] & 0xffffffffll);
                if (mbest[i] == (int)p && mbest[j] == (int)p) {
                    flag[p] = 2;
                    mmatch[i] = 1;
                    mmatch[j] = 1;
                }
            }
        __syncthreads();
        int live = 0;
        for (int64_t p = tid; p < np; p += T)
            if (flag[p] == 1) {
                const int i = (int)(keys[p] >> 32), j = (int)(keys[p] & 0xffffffffll);
                if (mmatch[i] || mmatch[j]) flag[p] = 0;
                else live = 1;
            }
        if (!__syncthreads_or(live)) break;
    }
    // impulses of the resolved pairs (disjoint moonlets): 1 = i, 2 = j
    for (int64_t p = tid; p < np; p += T) {
        if (flag[p] != 2) continue;
        const int i = (int)(keys[p] >> 32), j = (int)(keys[p] & 0xffffffffll);
        const double t = dtc[p];
        const double x1 = x[i] + t * vx[i], y1 = y[i] + t * vy[i], z1 = z[i] + t * vz[i];
        const double x2 = x[j] + t * vx[j], y2 = y[j] + t * vy[j], z2 = z[j] + t * vz[j];
        const double drx = x1 - x2, dry = y1 - y2, drz = z1 - z2;
        const double dvx = vx[i] - vx[j], dvy = vy[i] - vy[j], dvz = vz[i] - vz[j];
        const double sdot = drx * dvx + dry * dvy + drz * dvz;
        const double Rs = R[i] + R[j];
        const double alpha = f * m[i] * m[j] / ((m[i] + m[j]) * (Rs * Rs));
        const double Jx = alpha * sdot * drx, Jy = alpha * sdot * dry, Jz = alpha * sdot * drz;
        const double u1x = vx[i] - Jx / m[i], u1y = vy[i] - Jy / m[i], u1z = vz[i] - Jz / m[i];
        const double u2x = vx[j] + Jx / m[j], u2y = vy[j] + Jy / m[j], u2z = vz[j] + Jz / m[j];
        // old velocity up to contact, new one after: the drift adds dt u
        x[i] = x[i] + t * (vx[i] - u1x); y[i] = y[i] + t * (vy[i] - u1y);
        z[i] = z[i] + t * (vz[i] - u1z);
        x[j] = x[j] + t * (vx[j] - u2x); y[j] = y[j] + t * (vy[j] - u2y);
        z[j] = z[j] + t * (vz[j] - u2z);
        vx[i] = u1x; vy[i] = u1y; vz[i] = u1z;
        vx[j] = u2x; vy[j] = u2y; vz[j] = u2z;
    }
    // the resolved pairs, in (i, j) order, as (step, i, j) after the earlier steps'
    if (tid == 0) { s_run = 0; s_base = *cursor; }
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int64_t c0 = 0; c0 < np; c0 += T) {
        const int64_t p = c0 + tid;
        const bool acc = p < np && flag[p] == 2;
        const uint64_t b = __ballot(acc);
        if (lane == 0) wsum[w] = __popcll(b);
        __syncthreads();
        int before = 0, tot = 0;
        for (int k = 0; k < T / kWave; k++) {
            if (k < w) before += wsum[k];
            tot += wsum[k];
        }
        if (acc) {
            const int64_t o = s_base + s_run + before + __popcll(b & lt);
            if (o < cap) {
                pairs[3 * o] = step;
                pairs[3 * o + 1] = keys[p] >> 32;
                pairs[3 * o + 2] = keys[p] & 0xffffffffll;
            }
        }
        __syncthreads();
        if (tid == 0) s_run += tot;
        __syncthreads();
    }
    if (tid == 0) {
        *n_pairs_dev = s_run;
        if (s_base + s_run > cap) {
            atomicOr(&st->status, (int32_t)ST_CAP_PAIRS);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)(s_base + s_run));
        }
        *cursor = s_base + s_run;
    }
}

hipError_t launch_resolve(const Workspace &ws, double *x, double *y, double *z, double *vx,
                          double *vy, double *vz, const double *m, const double *R, double dt,
                          double f, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev, int step,
                          int64_t *cursor, hipStream_t s) {
    k_rank_pairs<<<256, 256, 0, s>>>(ws.st, ws.pairs_tmp, ws.pair_cap, ws.pairs_alt);
    k_resolve<<<1, kResolveThreads, 0, s>>>(ws.st, ws.pairs_alt, ws.pair_cap, x, y, z, vx, vy,
                                            vz, m, R, dt, f, ws.pair_dt, ws.pair_flag, ws.mbest,
                                            ws.mmatch, pairs, cap, n_pairs_dev, step, cursor);
    return hipGetLastError();
}

hipError_t launch_collide_pairs(const Workspace &ws, int64_t n, double dt, hipStream_t s) {
    (void)n;
    k_collide_init<<<1, 64, 0, s>>>(ws.st);
    k_collide<<<16384, 64, 0, s>>>(ws.st, ws.cand, ws.p2p_cap, ws.c_first, ws.c_count, ws.ccell,
                                   ws.xs, ws.ys, ws.zs, ws.vxs, ws.vys, ws.vzs, ws.rads, ws.idx,
                                   ws.pcol, dt, ws.pairs_tmp, ws.pair_cap, ws.count_part);
    return launch_sum_u64(ws.count_part, 16384, (unsigned long long *)&ws.st->col_tests, true,
                          s);
}

hipError_t launch_emit_pairs(const Workspace &ws, int64_t *pairs, int64_t cap,
                             int64_t *n_pairs_dev, int triple, int step, int64_t *cursor,
                             hipStream_t s) {
    k_rank_pairs<<<256, 256, 0, s>>>(ws.st, ws.pairs_tmp, ws.pair_cap, ws.pairs_alt);
    k_emit_pairs<<<256, 256, 0, s>>>(ws.st, ws.pairs_alt, ws.pair_cap, pairs, cap, n_pairs_dev,
                                     triple, step, cursor);
    k_pairs_done<<<1, 64, 0, s>>>(ws.st, n_pairs_dev, cap, ws.pair_cap, triple, cursor);
    return hipGetLastError();
}

}  // namespace ncorp

// Collision search on the candidate cell pairs of the collision walk (Alg. 2 with
// "do nothing" for well-separated cells) and the pair test of Sect. 3.1:
//   Delta = (dr.dv)^2 + dv^2 [(R1 + R2)^2 - dr^2]                      (Eq. 1)
//   dt_c  = -(dr.dv + sqrt(Delta)) / dv^2, collision iff 0 <= dt_c <= dt (Eq. 2)
// The arithmetic is FP64 with a fixed operation order and no contraction, and it is
// symmetric under swapping the two moonlets bit for bit (dr and dv only change
// sign), so the pair set is reproducible exactly.
#include "contact.h"

namespace ncorp {

// Value of lane `src` (the same for every lane of the wave) on all lanes: scalar
// reads, where a general shuffle would go through LDS permutes.
__device__ __forceinline__ int bcast_i(int v, int src) {
    return __builtin_amdgcn_readlane(v, src);
}
__device__ __forceinline__ double bcast_d(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double4 bcast4(double4 v, int src) {
    return make_double4(bcast_d(v.x, src), bcast_d(v.y, src), bcast_d(v.z, src),
                        bcast_d(v.w, src));
}

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
    double x, y, z, vx, vy, vz, R, reach;    // reach = R + dt |v|
    uint32_t id;
};

// A pair that touches at a time t in [0, dt] starts at most R_a + R_b + dt |v_a - v_b|
// <= reach_a + reach_b apart: the cheap distance check rejects nearly every pair before
// Eqs. (1)-(2) are evaluated (relative margin 1e-9, far above rounding).
__device__ __forceinline__ bool within_reach(const PState &a, const PState &b) {
    const double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    const double rs = a.reach + b.reach;
    return dx * dx + dy * dy + dz * dz <= rs * rs * (1.0 + 1e-9);
}

__device__ __forceinline__ void test_pair(const PState &p, const PState &o, double dt,
                                          int64_t *out, int64_t cap, DevState *st) {
    if (within_reach(p, o) &&
        pair_test(p.x, p.y, p.z, p.vx, p.vy, p.vz, p.R, o.x, o.y, o.z, o.vx, o.vy, o.vz, o.R, dt))
        record(out, cap, (unsigned long long *)&st->npairs, p.id, o.id);
}

// Can moonlet p = (x, y, z, R + dt |v|) meet a moonlet of the other cell within the
// step?  A pair that touches at a time t in [0, dt] starts at most R_a + R_b +
// dt (|v_a| + |v_b|) apart.  Spheres (BOXES = false, from the collision climb): the
// other cell's moonlets lie within r_crit - (R + dt |v|) of its centre, so
// |r_a - s| <= R_a + dt |v_a| + r_crit (a = centre, radius).  Boxes (BOXES = true):
// the other leaf's moonlets lie in the box [a.xyz, b.xyz], each with a reach of at
// most a.w, so the distance from r_a to the box is at most R_a + dt |v_a| + a.w.
// The relative margin 1e-9 dwarfs the rounding of either side, so no pair the exact
// test accepts is dropped.
template <bool BOXES>
__device__ __forceinline__ bool can_reach(const double4 &p, const double4 &a, const double4 &b) {
    if (BOXES) {
        const double gx = fmax(0.0, fmax(a.x - p.x, p.x - b.x));
        const double gy = fmax(0.0, fmax(a.y - p.y, p.y - b.y));
        const double gz = fmax(0.0, fmax(a.z - p.z, p.z - b.z));
        const double rs = p.w + a.w;
        return gx * gx + gy * gy + gz * gz <= rs * rs * (1.0 + 1e-9);
    }
    const double reach = p.w + a.w;
    const double dx = p.x - a.x, dy = p.y - a.y, dz = p.z - a.z;
    return dx * dx + dy * dy + dz * dz <= reach * reach * (1.0 + 1e-9);
}

// Moonlets of cell C (first f, count n) that can reach the other cell within the
// step (can_reach).  The survivors are compacted into out[] in moonlet order;
// returns their number, or -1 if more than `limit` survive.
template <bool BOXES>
__device__ __forceinline__ int cull_cell(int f, int n, double4 oa, double4 ob,
                                         const double4 *__restrict__ pcol,
                                         const double4 *__restrict__ vcol,
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
            // position and R + dt |v|, as the climb or the box pass stored them
            const double4 p = pcol[k];
            ps.x = p.x; ps.y = p.y; ps.z = p.z; ps.reach = p.w;
            keep = can_reach<BOXES>(p, oa, ob);
        }
        if (keep) {
            const double4 v = vcol[k];
            ps.vx = v.x; ps.vy = v.y; ps.vz = v.z; ps.R = v.w;
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

// All pairs of one cell of n <= 64 moonlets staged in sb: (i, i + d mod n) for
// d = 1 .. n/2 (for even n, d = n/2 only from i < n/2) is every unordered pair once.
// Lane groups of S >= n lanes take different d, so the rounds stay full instead of
// shrinking as i grows.
__device__ __forceinline__ void self_pairs_staged(int n, const PState *sb,
                                                  const double4 *spos, double dt,
                                                  int64_t *out, int64_t cap, DevState *st,
                                                  unsigned long long &tests) {
    const int lane = threadIdx.x;
    int S = 1;
    while (S < n) S <<= 1;
    const int G = kWave / S, i = lane % S, grp = lane / S, dmax = n / 2;
    if (i >= n) return;
    const PState me = sb[i];
    for (int d0 = 1; d0 <= dmax; d0 += G) {
        const int d = d0 + grp;
        if (d > dmax || (2 * d == n && i >= d)) continue;
        int j = i + d;
        if (j >= n) j -= n;
        tests++;
        const double4 o = spos[j];
        const double dx = me.x - o.x, dy = me.y - o.y, dz = me.z - o.z;
        const double rs = me.reach + o.w;
        if (dx * dx + dy * dy + dz * dz <= rs * rs * (1.0 + 1e-9)) test_pair(me, sb[j], dt, out, cap, st);
    }
}

// Every moonlet pair of the candidate cell pair (A, B) (i < j when A == B): lanes
// take moonlets of A, B's moonlets are staged in LDS 64 at a time and split over
// lane groups when A holds fewer than 64.
__device__ __forceinline__ void test_cell_pair(
    int2 pr, PState *sb, double4 *spos, const int32_t *__restrict__ c_first,
    const int32_t *__restrict__ c_count, const uint32_t *__restrict__ perm,
    const double4 *__restrict__ pcol, const double4 *__restrict__ vcol, double dt, int64_t *out,
    int64_t cap, DevState *st, unsigned long long &tests) {
    const int lane = threadIdx.x;
    const int fa = c_first[pr.x], na = c_count[pr.x];
    const int fb = c_first[pr.y], nb = c_count[pr.y];
    const bool self = pr.x == pr.y;
    if (self && na <= kWave) {
        __syncthreads();
        if (lane < na) {
            const int b = fa + lane;
            PState ps;
            const double4 p = pcol[b], v = vcol[b];
            ps.x = p.x; ps.y = p.y; ps.z = p.z; ps.reach = p.w;
            ps.vx = v.x; ps.vy = v.y; ps.vz = v.z; ps.R = v.w;
            ps.id = perm[b];
            sb[lane] = ps;
            spos[lane] = p;
        }
        __syncthreads();
        self_pairs_staged(na, sb, spos, dt, out, cap, st, tests);
        return;
    }
    for (int a0 = 0; a0 < na; a0 += 64) {
        const int nac = na - a0 < 64 ? na - a0 : 64;
        int S = 1;
        while (S < nac) S <<= 1;
        const int G = 64 / S, tl = lane % S, grp = lane / S;
        const bool act = tl < nac;
        const int ia = a0 + (act ? tl : 0);
        const int a = fa + ia;
        PState me;
        {
            const double4 p = pcol[a], v = vcol[a];
            me.x = p.x; me.y = p.y; me.z = p.z; me.reach = p.w;
            me.vx = v.x; me.vy = v.y; me.vz = v.z; me.R = v.w;
        }
        me.id = perm[a];
        for (int b0 = self ? a0 : 0; b0 < nb; b0 += 64) {
            const int nbc = nb - b0 < 64 ? nb - b0 : 64;
            __syncthreads();
            if (lane < nbc) {
                const int b = fb + b0 + lane;
                PState ps;
                const double4 p = pcol[b], v = vcol[b];
                ps.x = p.x; ps.y = p.y; ps.z = p.z; ps.reach = p.w;
                ps.vx = v.x; ps.vy = v.y; ps.vz = v.z; ps.R = v.w;
                ps.id = perm[b];
                sb[lane] = ps;
            }
            __syncthreads();
            if (!act) continue;
            const int jlo = self ? (ia + 1 - b0 > 0 ? ia + 1 - b0 : 0) : 0;
            // first j >= jlo with j = grp (mod G)
            int j = jlo + ((grp - jlo % G) % G + G) % G;
            for (; j < nbc; j += G) {
                tests++;
                test_pair(me, sb[j], dt, out, cap, st);
            }
        }
    }
}

// candidate slots a wave reads at a time; the cell ranges and spheres of both
// sides of all of them are loaded in one go
constexpr int kCandRound = 8;

// BOXES: the candidates are leaf pairs with bounding boxes (cbox: low corner and
// largest reach, high corner, per cell); otherwise cell pairs with the collision
// climb's spheres (ccell).
template <bool BOXES>
__global__ void __launch_bounds__(64)
k_collide(DevState *st, const int2 *__restrict__ cand, int64_t cand_cap,
          const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
          const double4 *__restrict__ ccell, const double4 *__restrict__ cbox,
          const uint32_t *__restrict__ perm, const double4 *__restrict__ pcol,
          const double4 *__restrict__ vcol, const int32_t *__restrict__ ent_cell, double dt,
          int64_t *out, int64_t cap, unsigned long long *tests_part) {
    __shared__ PState sp[kWave];    // survivors of both sides (or a staged tile of B)
    __shared__ double4 spos[kWave];
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
        double4 sph = make_double4(0.0, 0.0, 0.0, 0.0), shi = sph;
        if (side) {
            cf = c_first[mine];
            cn = c_count[mine];
            if (BOXES) {
                sph = cbox[2 * (int64_t)other];
                shi = cbox[2 * (int64_t)other + 1];
            } else {
                sph = ccell[other];
            }
        }
        uint64_t live = __ballot(lane < kCandRound && cq.x >= 0);   // gaps are skipped
        while (live) {
            const int l = __ffsll((unsigned long long)live) - 1;
            live &= live - 1;
            const int2 pr = make_int2(bcast_i(cq.x, l), bcast_i(cq.y, l));
            if (pr.x != pr.y) {
                // distinct cells: keep only moonlets that can reach the other cell
                const int lb = kCandRound + l;
                const int fa = bcast_i(cf, l), na = bcast_i(cn, l);
                const int fb = bcast_i(cf, lb), nb = bcast_i(cn, lb);
                int ka = -1, kb = -1;
                __syncthreads();
                if (BOXES && na + nb <= 2 * kWave) {
                    // both sides at once, two moonlets per lane (item t = lane, lane + 64
                    // is A[t] for t < na, else B[t - na]), whole records loaded together:
                    // one dependent round trip per candidate
                    const double4 oA = bcast4(sph, l), hA = bcast4(shi, l);
                    const double4 oB = bcast4(sph, lb), hB = bcast4(shi, lb);
                    PState ps[2];
                    bool keep[2], isA[2];
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const int t = lane + u * kWave;
                        isA[u] = t < na;
                        keep[u] = false;
                        if (t < na + nb) {
                            const int k = isA[u] ? fa + t : fb + (t - na);
                            const double4 p = pcol[k], v = vcol[k];
                            ps[u].x = p.x; ps[u].y = p.y; ps[u].z = p.z; ps[u].reach = p.w;
                            ps[u].vx = v.x; ps[u].vy = v.y; ps[u].vz = v.z; ps[u].R = v.w;
                            ps[u].id = perm[k];
                            // an A moonlet is culled against B's box and the other way round
                            keep[u] = isA[u] ? can_reach<true>(p, oA, hA)
                                             : can_reach<true>(p, oB, hB);
                        }
                    }
                    const uint64_t mA0 = __ballot(keep[0] && isA[0]);
                    const uint64_t mA1 = __ballot(keep[1] && isA[1]);
                    const uint64_t mB0 = __ballot(keep[0] && !isA[0]);
                    const uint64_t mB1 = __ballot(keep[1] && !isA[1]);
                    const int a0 = __popcll(mA0), b0 = __popcll(mB0);
                    ka = a0 + __popcll(mA1);
                    kb = b0 + __popcll(mB1);
                    if (ka + kb <= kWave) {
                        if (keep[0])
                            sp[isA[0] ? __popcll(mA0 & lt) : ka + __popcll(mB0 & lt)] = ps[0];
                        if (keep[1])
                            sp[isA[1] ? a0 + __popcll(mA1 & lt) : ka + b0 + __popcll(mB1 & lt)] =
                                ps[1];
                    } else {
                        ka = kb = -1;
                    }
                } else if (na + nb <= kWave) {
                    // both sides in one round: lanes [0, na) hold A, [na, na + nb) hold B
                    const bool inA = lane < na, inB = !inA && lane < na + nb;
                    const int sl = inA ? l : lb;
                    const double4 s4 = make_double4(__shfl(sph.x, sl), __shfl(sph.y, sl),
                                                    __shfl(sph.z, sl), __shfl(sph.w, sl));
                    double4 h4 = s4;
                    if (BOXES)
                        h4 = make_double4(__shfl(shi.x, sl), __shfl(shi.y, sl),
                                          __shfl(shi.z, sl), 0.0);
                    bool keep = false;
                    int k = 0;
                    double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
                    if (inA || inB) {
                        k = inA ? fa + lane : fb + (lane - na);
                        p = pcol[k];
                        keep = can_reach<BOXES>(p, s4, h4);
                    }
                    const uint64_t mA = __ballot(keep && inA), mB = __ballot(keep && inB);
                    ka = __popcll(mA);
                    kb = __popcll(mB);
                    if (keep) {
                        PState ps;
                        ps.x = p.x; ps.y = p.y; ps.z = p.z; ps.reach = p.w;
                        const double4 v = vcol[k];
                        ps.vx = v.x; ps.vy = v.y; ps.vz = v.z; ps.R = v.w;
                        ps.id = perm[k];
                        sp[inA ? __popcll(mA & lt) : ka + __popcll(mB & lt)] = ps;
                    }
                } else {
                    const double4 sA = bcast4(sph, l), sB = bcast4(sph, lb);
                    const double4 hA = bcast4(shi, l), hB = bcast4(shi, lb);
                    ka = cull_cell<BOXES>(fa, na, sA, hA, pcol, vcol, perm, sp, kWave);
                    kb = ka < 0 ? -1
                                : cull_cell<BOXES>(fb, nb, sB, hB, pcol, vcol, perm, sp + ka,
                                                   kWave - ka);
                }
                __syncthreads();
                if (ka >= 0 && kb >= 0) {
                    const int tot = ka * kb;
                    for (int t = lane; t < tot; t += kWave) {
                        tests++;
                        test_pair(sp[t / kb], sp[ka + t % kb], dt, out, cap, st);
                    }
                    continue;
                }
            }
            test_cell_pair(pr, sp, spos, c_first, c_count, perm, pcol, vcol, dt, out, cap, st,
                           tests);
        }
    }
    if (BOXES) {
        // then every leaf with itself (the candidates hold distinct leaves only); blocks
        // that finish their candidates early start here, so both kinds of work overlap
        const int K = st->nleaves;
        for (int e = blockIdx.x; e < K; e += gridDim.x) {
            const int c = ent_cell[e];
            const int n = c_count[c];
            if (n < 2) continue;
            if (n > kWave) {
                test_cell_pair(make_int2(c, c), sp, spos, c_first, c_count, perm, pcol, vcol, dt,
                               out, cap, st, tests);
                continue;
            }
            __syncthreads();
            if (lane < n) {
                const int k = c_first[c] + lane;
                const double4 p = pcol[k], v = vcol[k];
                PState ps;
                ps.x = p.x; ps.y = p.y; ps.z = p.z; ps.reach = p.w;
                ps.vx = v.x; ps.vy = v.y; ps.vz = v.z; ps.R = v.w;
                ps.id = perm[k];
                sp[lane] = ps;
                spos[lane] = p;
            }
            __syncthreads();
            self_pairs_staged(n, sp, spos, dt, out, cap, st, tests);
        }
    }
    // per-block partials, summed by the pair ranking that follows: one atomic per wave
    // on a single counter would serialise all blocks of the grid
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

// Rank sort of the (distinct) pair keys: rank = number of smaller keys.  A block of
// kRankSplit waves takes 64 keys (a lane each); wave w counts the smaller keys in the
// w-th of kRankSplit equal segments of the list, walking it in chunks of 256 keys
// loaded coalesced (the next chunk while the current one is compared) and read back
// from LDS as wave-wide broadcasts; the block then adds the counts of its waves.
constexpr int kRankSplit = 8;
constexpr int kRankGrid = 2048;
constexpr int kRankSumBlocks = 16;   // blocks that also add up the pair-test counts
constexpr int kRankChunk = 4 * kWave;
// The resolution's per-pair start (when dtc is non-null): contact time (Eq. 2) of
// every ranked pair at its rank, its live flag, and its moonlets' matched flags cleared
struct RankResolve {
    const double *x, *y, *z, *vx, *vy, *vz, *R;
    double dt;
    double *dtc;
    int32_t *flag, *mmatch;
};

__global__ void __launch_bounds__(kWave * kRankSplit)
k_rank_pairs(DevState *__restrict__ st, const int64_t *__restrict__ in, int64_t cap,
             int64_t *__restrict__ out, const unsigned long long *__restrict__ tests_part,
             int n_part, const RankResolve RR) {
    __shared__ int64_t tile_all[kRankSplit][kRankChunk];
    __shared__ int64_t part[kRankSplit][kWave];
    const int sum_b = (int)blockIdx.x - ((int)gridDim.x - kRankSumBlocks);
    if (tests_part && sum_b >= 0) {
        // the pair tests' per-block counts, summed by the last kRankSumBlocks blocks
        // (which have no keys to rank unless the list is long), one integer atomic each
        const int per = (n_part + kRankSumBlocks - 1) / kRankSumBlocks;
        const int i0 = sum_b * per, i1 = i0 + per < n_part ? i0 + per : n_part;
        unsigned long long v = 0;
        for (int i = i0 + threadIdx.x; i < i1; i += blockDim.x) v += tests_part[i];
        for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
        unsigned long long *red = (unsigned long long *)&part[0][0];
        __syncthreads();
        if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (int k = 0; k < (int)blockDim.x / kWave; k++) t += red[k];
            atomicAdd((unsigned long long *)&st->col_tests, t);
        }
        __syncthreads();
    }
    int64_t n = st->npairs;
    // the resolution takes no pair of an overflowed list or after a failed pass
    const bool resolve = RR.dtc && n <= cap && !(st->status & kSkipMask);
    if (n > cap) n = cap;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int64_t *tile = tile_all[w];
    // this wave's segment of the list
    const int64_t seg = (n + kRankSplit - 1) / kRankSplit;
    const int64_t s0 = seg * w < n ? seg * w : n;
    const int64_t s1 = s0 + seg < n ? s0 + seg : n;
    for (int64_t base = (int64_t)blockIdx.x * kWave; base < n; base += (int64_t)gridDim.x * kWave) {
        const int64_t i = base + lane;
        const int64_t v = i < n ? in[i] : INT64_MAX;
        int64_t r0 = 0, r1 = 0;
        int64_t nxt[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int64_t q = s0 + u * kWave + lane;
            nxt[u] = q < s1 ? in[q] : INT64_MAX;
        }
        for (int64_t t0 = s0; t0 < s1; t0 += kRankChunk) {
            wave_sync();
#pragma unroll
            for (int u = 0; u < 4; u++) tile[u * kWave + lane] = nxt[u];
            wave_sync();
            const int64_t t1 = t0 + kRankChunk;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int64_t q = t1 + u * kWave + lane;
                nxt[u] = q < s1 ? in[q] : INT64_MAX;
            }
            // padding keys (INT64_MAX) are never below a real key
#pragma unroll 8
            for (int k = 0; k < kRankChunk; k += 2) {
                r0 += tile[k] < v;
                r1 += tile[k + 1] < v;
            }
        }
        part[w][lane] = r0 + r1;
        __syncthreads();
        if (w == 0 && i < n) {
            int64_t r = 0;
#pragma unroll
            for (int k = 0; k < kRankSplit; k++) r += part[k][lane];
            out[r] = v;
            if (resolve) {
                const int a = (int)(v >> 32), b = (int)(v & 0xffffffffll);
                const double t = contact_time(RR.x[a], RR.y[a], RR.z[a], RR.vx[a], RR.vy[a],
                                              RR.vz[a], RR.R[a], RR.x[b], RR.y[b], RR.z[b],
                                              RR.vx[b], RR.vy[b], RR.vz[b], RR.R[b], RR.dt);
                RR.dtc[r] = t;
                RR.flag[r] = t >= 0.0 ? 1 : 0;
                RR.mmatch[a] = 0;
                RR.mmatch[b] = 0;
            }
        }
        __syncthreads();
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
// ---------------------------------------------------------------- candidates from lists
// Collision candidates from the gravity walk's lists of the same tree (well-separated
// cell pairs, direct-sum cell pairs, direct-sum self cells).  Those lists cover every
// moonlet pair exactly once, so the leaf pairs below their interactions, minus those
// that provably cannot collide, are candidates covering every colliding pair once:
// the pair set is the collision walk's.  A pair that touches within the step starts
// at most R_a + R_b + dt (|v_a| + |v_b|) apart, so two cells can hold a colliding pair
// only if their bounding boxes, each grown by its largest R + dt |v|, overlap.  A leaf's
// box is the tight box of its moonlets (k_leaf_boxes); an interaction with an internal
// cell is first tested on the gravity climb's spheres (cells_may_meet).  The pairs
// inside each leaf are searched apart from the candidates (by k_collide, after them).
struct CBox {
    double lx, ly, lz, hx, hy, hz, r;
};

__device__ __forceinline__ bool boxes_meet(const CBox &a, const CBox &b) {
    const double gx = fmax(0.0, fmax(b.lx - a.hx, a.lx - b.hx));
    const double gy = fmax(0.0, fmax(b.ly - a.hy, a.ly - b.hy));
    const double gz = fmax(0.0, fmax(b.lz - a.hz, a.lz - b.hz));
    const double rs = (a.r + b.r) * (1.0 + 1e-9);
    return gx * gx + gy * gy + gz * gz <= rs * rs;
}

__device__ __forceinline__ CBox leaf_box(const double4 *__restrict__ cbox, int c) {
    const double4 lo = cbox[2 * (int64_t)c], hi = cbox[2 * (int64_t)c + 1];
    return CBox{lo.x, lo.y, lo.z, hi.x, hi.y, hi.z, lo.w};
}

struct BoxArgs {
    const double4 *cbox;
    const double4 *gcell;         // gravity climb: centre of mass (x, y, z)
    const double *c_rmax;         // gravity climb: r_max (bounds every moonlet's distance)
};

// May cells a and b hold a colliding pair?  Their gravity climb spheres, grown by the
// largest reach of all moonlets, must overlap: every moonlet of a cell lies within
// r_max of its centre of mass (Eq. 11 and the corner clamp), so the pair's moonlets
// are at least |s_a - s_b| - r_max,a - r_max,b apart.  (The walk's well-separated
// pairs are far apart on that scale and drop here; the leaf pairs below the others
// are then tested on their boxes.)
__device__ __forceinline__ bool cells_may_meet(const BoxArgs &B, const DevState *st, int a,
                                               int b) {
    const double4 sa = B.gcell[a], sb = B.gcell[b];
    const double r = __longlong_as_double((long long)st->reach_max);
    const double dx = sa.x - sb.x, dy = sa.y - sb.y, dz = sa.z - sb.z;
    const double rs = (B.c_rmax[a] + B.c_rmax[b] + 2.0 * r) * (1.0 + 1e-9);
    return dx * dx + dy * dy + dz * dz <= rs * rs;
}

// Counts (out == nullptr) or writes the candidate leaf pairs of one interaction.
__device__ __forceinline__ int leaf_candidates(int2 pr, const BoxArgs &B, const DevState *st,
                                               const int32_t *__restrict__ c_entry,
                                               const int32_t *__restrict__ c_nent,
                                               const int32_t *__restrict__ c_count,
                                               const int32_t *__restrict__ ent_cell, int2 *out,
                                               int64_t pos, int64_t cap) {
    if (pr.x < 0) return 0;
    const bool self = pr.x == pr.y;
    if (!self && !cells_may_meet(B, st, pr.x, pr.y)) return 0;
    const int ea = c_entry[pr.x], na = c_nent[pr.x];
    const int eb = c_entry[pr.y], nb = c_nent[pr.y];
    int k = 0;
    for (int i = 0; i < na; i++) {
        const int la = ent_cell[ea + i];
        const CBox sa = leaf_box(B.cbox, la);
        // four leaves of B at a time: their loads are independent of each other
        for (int j0 = self ? i : 0; j0 < nb; j0 += 4) {
            int lb[4];
            CBox sb[4];
#pragma unroll
            for (int u = 0; u < 4; u++) lb[u] = j0 + u < nb ? ent_cell[eb + j0 + u] : la;
#pragma unroll
            for (int u = 0; u < 4; u++) sb[u] = leaf_box(B.cbox, lb[u]);
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (j0 + u >= nb) continue;
                // a leaf with itself is searched by k_collide after the candidates
                const bool take = la != lb[u] && boxes_meet(sa, sb[u]);
                if (!take) continue;
                if (out && pos + k < cap) out[pos + k] = make_int2(la, lb[u]);
                k++;
            }
        }
    }
    return k;
}

// One wave per leaf: every moonlet's (x, y, z, R + dt |v|) record for the culling, the
// tight box of the leaf's moonlets with their largest R + dt |v|, and the largest of
// all moonlets (for the cubes of internal cells).
__global__ void __launch_bounds__(kWave)
k_leaf_boxes(DevState *st, const double *__restrict__ xs, const double *__restrict__ ys,
             const double *__restrict__ zs, const double4 *__restrict__ pack4,
             const uint32_t *__restrict__ perm, double dt, const int32_t *__restrict__ ent_cell,
             const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
             double4 *__restrict__ cbox, double4 *__restrict__ pcol,
             double4 *__restrict__ vcol, unsigned long long *__restrict__ part) {
    if (st->status & kSkipMask) {
        if (threadIdx.x == 0) part[blockIdx.x] = 0ull;
        return;
    }
    const int K = st->nleaves;
    const int lane = threadIdx.x;
    double wmax = 0.0;
    for (int e = blockIdx.x; e < K; e += gridDim.x) {
        const int c = ent_cell[e];
        const int f = c_first[c], cnt = c_count[c];
        double lx = INFINITY, ly = INFINITY, lz = INFINITY;
        double hx = -INFINITY, hy = -INFINITY, hz = -INFINITY, ex = 0.0;
        for (int c0 = lane; c0 < cnt; c0 += kWave) {
            const int k = f + c0;
            const double x = xs[k], y = ys[k], z = zs[k];
            const double4 w = pack4[perm[k]];          // (vx, vy, vz, R), input order
            const double v = sqrt(w.x * w.x + w.y * w.y + w.z * w.z);
            const double ee = (w.w + dt * v) - 0.0;
            pcol[k] = make_double4(x, y, z, ee);
            vcol[k] = w;
            lx = fmin(lx, x); ly = fmin(ly, y); lz = fmin(lz, z);
            hx = fmax(hx, x); hy = fmax(hy, y); hz = fmax(hz, z);
            ex = fmax(ex, ee);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) {
            lx = fmin(lx, __shfl_xor(lx, o)); ly = fmin(ly, __shfl_xor(ly, o));
            lz = fmin(lz, __shfl_xor(lz, o));
            hx = fmax(hx, __shfl_xor(hx, o)); hy = fmax(hy, __shfl_xor(hy, o));
            hz = fmax(hz, __shfl_xor(hz, o));
            ex = fmax(ex, __shfl_xor(ex, o));
        }
        if (lane == 0) {
            cbox[2 * (int64_t)c] = make_double4(lx, ly, lz, ex);
            cbox[2 * (int64_t)c + 1] = make_double4(hx, hy, hz, 0.0);
        }
        wmax = fmax(wmax, ex);
    }
    // per-block partial maxima (reaches are >= 0, so their bit patterns order like the
    // values); one atomic per block on a single word would serialise the grid
    if (lane == 0) part[blockIdx.x] = (unsigned long long)__double_as_longlong(wmax);
}

// st->reach_max = the largest of the n partials
__global__ void __launch_bounds__(1024)
k_max_u64(const unsigned long long *__restrict__ part, int64_t n, DevState *st) {
    __shared__ unsigned long long red[1024 / kWave];
    // the box pass precedes every search on the gravity lists: the pair and test
    // counts of that search start here
    if (threadIdx.x == 0) { st->npairs = 0; st->col_tests = 0; }
    unsigned long long v = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) v = part[i] > v ? part[i] : v;
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int k = 0; k < 1024 / kWave; k++) t = red[k] > t ? red[k] : t;
        st->reach_max = t;
    }
}

constexpr int kBoxGrid = 16384;

hipError_t launch_leaf_boxes(const Workspace &ws, int64_t n, double dt, hipStream_t s) {
    (void)n;
    k_leaf_boxes<<<kBoxGrid, kWave, 0, s>>>(ws.st, ws.xs, ws.ys, ws.zs, ws.pack4, ws.idx, dt,
                                            ws.ent_cell, ws.c_first, ws.c_count,
                                            ws.cbox, ws.pcol, ws.vcol, ws.count_part);
    k_max_u64<<<1, 1024, 0, s>>>(ws.count_part, kBoxGrid, ws.st);
    return hipGetLastError();
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
             const int2 *__restrict__ p2p, int64_t p2p_cap, const BoxArgs B,
             const int32_t *__restrict__ c_entry, const int32_t *__restrict__ c_nent,
             const int32_t *__restrict__ c_count, const int32_t *__restrict__ ent_cell,
             int32_t *__restrict__ blk, uint64_t *__restrict__ live_bits) {
    __shared__ int wtot[kCandBlock / kWave];
    const CandLists L = cand_lists(st, m2l, m2l_cap, p2p, p2p_cap);
    const bool skip = (st->status & kSkipMask) != 0;
    int sum = 0;
    for (int64_t q0 = (int64_t)blockIdx.x * kCandBlock; q0 < L.total && !skip;
         q0 += (int64_t)gridDim.x * kCandBlock) {
        const int64_t q = q0 + threadIdx.x;
        int2 pr = make_int2(-1, -1);
        if (q < L.total) pr = q < L.nm ? L.m2l[q] : L.p2p[q - L.nm];   // gaps are (-1, -1)
        const int cnt = leaf_candidates(pr, B, st, c_entry, c_nent, c_count, ent_cell, nullptr,
                                        0, 0);
        // one bit per slot with candidates (a wave's 64 slots are one aligned word)
        if (live_bits) {
            const uint64_t m = __ballot(cnt > 0);
            if ((threadIdx.x & (kWave - 1)) == 0) live_bits[(q0 + threadIdx.x) / kWave] = m;
        }
        int excl;
        sum += block_excl(cnt, excl, wtot);
    }
    if (threadIdx.x == 0) blk[blockIdx.x] = sum;
}

// exclusive scan of the block counts (one block); the total is the candidate count
__global__ void __launch_bounds__(1024) k_cand_scan(DevState *st, int32_t *blk, int nb) {
    __shared__ int32_t wtot[1024 / kWave];
    constexpr int kPer = 8;          // consecutive counts per thread: one round up to 8192
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int32_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 1024 * kPer) {
        const int i0 = b0 + threadIdx.x * kPer;
        int32_t x[kPer], sum = 0;
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            x[u] = i0 + u < nb ? blk[i0 + u] : 0;
            sum += x[u];
        }
        int32_t v = sum;
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
        int32_t run = carry + before + v - sum;
#pragma unroll
        for (int u = 0; u < kPer; u++) {
            if (i0 + u < nb) blk[i0 + u] = run;
            run += x[u];
        }
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
             const int2 *__restrict__ p2p, int64_t p2p_cap, const BoxArgs B,
             const int32_t *__restrict__ c_entry, const int32_t *__restrict__ c_nent,
             const int32_t *__restrict__ c_count, const int32_t *__restrict__ ent_cell,
             const int32_t *__restrict__ blk, int2 *cand, int64_t cand_cap,
             const uint64_t *__restrict__ live_bits) {
    __shared__ int wtot[kCandBlock / kWave];
    if (st->status & kSkipMask) return;
    const CandLists L = cand_lists(st, m2l, m2l_cap, p2p, p2p_cap);
    int64_t run = blk[blockIdx.x];
    for (int64_t q0 = (int64_t)blockIdx.x * kCandBlock; q0 < L.total;
         q0 += (int64_t)gridDim.x * kCandBlock) {
        const int64_t q = q0 + threadIdx.x;
        // the count pass's bits: slots without candidates need no second look
        const bool live = !live_bits ||
                          ((live_bits[(q0 + threadIdx.x) / kWave] >> (threadIdx.x & (kWave - 1))) & 1ull);
        int2 pr = make_int2(-1, -1);
        if (q < L.total && live) pr = q < L.nm ? L.m2l[q] : L.p2p[q - L.nm];
        const int cnt = leaf_candidates(pr, B, st, c_entry, c_nent, c_count, ent_cell, nullptr,
                                        0, 0);
        int excl;
        const int all = block_excl(cnt, excl, wtot);
        const int64_t pos = run + excl;
        if (cnt) leaf_candidates(pr, B, st, c_entry, c_nent, c_count, ent_cell, cand, pos,
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
    BoxArgs B;
    B.cbox = ws.cbox;
    B.gcell = ws.gcell;
    B.c_rmax = ws.c_rmax;
    // one bit per list slot in the tree-order direct sums' buffer (3n words, free during
    // a collision search), where the slots fit
    const int64_t words = (ws.m2l_cap + ws.p2p_cap + kWave - 1) / kWave + kCandBlock / kWave;
    uint64_t *bits = words <= 3 * ws.n_max ? (uint64_t *)ws.acc_s : nullptr;
    k_cand_count<<<(int)g, kCandBlock, 0, s>>>(ws.st, ws.m2l, ws.m2l_cap, ws.p2p, ws.p2p_cap, B,
                                               ws.c_entry, ws.c_nent, ws.c_count, ws.ent_cell,
                                               ws.cand_blk, bits);
    k_cand_scan<<<1, 1024, 0, s>>>(ws.st, ws.cand_blk, (int)g);
    k_cand_write<<<(int)g, kCandBlock, 0, s>>>(ws.st, ws.m2l, ws.m2l_cap, ws.p2p, ws.p2p_cap, B,
                                               ws.c_entry, ws.c_nent, ws.c_count, ws.ent_cell,
                                               ws.cand_blk, ws.cand, ws.p2p_cap, bits);
    return hipGetLastError();
}

// ---------------------------------------------------------------- resolution
// Hard-sphere resolution of the pairs found (Sect. 5.1-5.2), one block.  Pairs are
// taken in increasing (dt_c, i, j) and a moonlet collides at most once per step:
// this greedy matching is reached in rounds, each accepting every live pair that
// is the earliest live pair of both its moonlets (the earliest live pair of all is
// always one, so every round makes progress) and dropping the live pairs that
// touch a moonlet just matched -- the same set as taking the pairs one by one.
// Each round visits only the pairs still live.
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
constexpr int kResolveGrid = 512;      // blocks of the per-pair passes

// exclusive prefix of v >= 0 over the block (wsum: one word per wave), and the
// block's total
__device__ __forceinline__ int block_int_prefix(int v, int *wsum, int *total) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    int before = 0, tot = 0;
    for (int k = 0; k < (int)blockDim.x / kWave; k++) {
        if (k < w) before += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

__device__ __forceinline__ int pair_i(int64_t key) { return (int)(key >> 32); }
__device__ __forceinline__ int pair_j(int64_t key) { return (int)(key & 0xffffffffll); }

// pairs per thread and pass of the one-block rounds
constexpr int kResolveUnroll = 4;

// number of pairs the resolution takes: 0 when the list overflowed (the status then
// says so) or an earlier pass failed
__device__ __forceinline__ int resolve_count(const DevState *st, int64_t pair_cap) {
    const int64_t np = st->npairs;
    if (np > pair_cap || (st->status & kSkipMask)) return 0;
    return (int)np;                       // pair indices are 32-bit (the capacity is)
}

// The rounds of the matching and the list of resolved pairs, one block.
__global__ void __launch_bounds__(kResolveThreads)
k_resolve(DevState *st, const int64_t *__restrict__ keys, int64_t pair_cap,
          const double *__restrict__ dtc, int32_t *flag, int32_t *mbest, int32_t *mmatch,
          int32_t *live, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev, int step,
          int64_t *cursor) {
    constexpr int U = kResolveUnroll;
    __shared__ int wsum[kResolveThreads / kWave];
    const int tid = threadIdx.x;
    const int T = blockDim.x;
    if (st->npairs > pair_cap && !(st->status & kSkipMask) && tid == 0) {
        // the list is incomplete: nothing is resolved
        atomicOr(&st->status, (int32_t)ST_CAP_PAIRS);
        atomicMax((unsigned long long *)&st->required, (unsigned long long)st->npairs);
    }
    const int np = resolve_count(st, pair_cap);
    // flag: 0 dropped, 1 live, 2 resolved; the live pairs' indices are kept compacted
    // in `live`, so later rounds visit only what is left
    int nlive = 0;
    for (int c0 = 0; c0 < np; c0 += U * T) {
        int cnt = 0;
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int p = c0 + U * tid + u;
            ok[u] = p < np && flag[p] == 1;
            cnt += ok[u] ? 1 : 0;
        }
        int tot;
        int o = nlive + block_int_prefix(cnt, wsum, &tot);
#pragma unroll
        for (int u = 0; u < U; u++)
            if (ok[u]) live[o++] = c0 + U * tid + u;
        nlive += tot;
    }
    __syncthreads();
    while (nlive > 0) {
        for (int c0 = 0; c0 < nlive; c0 += U * T)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int q = c0 + u * T + tid;
                if (q < nlive) {
                    const int64_t k = keys[live[q]];
                    mbest[pair_i(k)] = -1;
                    mbest[pair_j(k)] = -1;
                }
            }
        __syncthreads();
        for (int c0 = 0; c0 < nlive; c0 += U * T)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int q = c0 + u * T + tid;
                if (q < nlive) {
                    const int p = live[q];
                    const int64_t k = keys[p];
                    keep_earliest(&mbest[pair_i(k)], p, dtc);
                    keep_earliest(&mbest[pair_j(k)], p, dtc);
                }
            }
        __syncthreads();
        for (int c0 = 0; c0 < nlive; c0 += U * T)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int q = c0 + u * T + tid;
                if (q < nlive) {
                    const int p = live[q];
                    const int64_t k = keys[p];
                    const int i = pair_i(k), j = pair_j(k);
                    if (mbest[i] == p && mbest[j] == p) {
                        flag[p] = 2;
                        mmatch[i] = 1;
                        mmatch[j] = 1;
                    }
                }
            }
        __syncthreads();
        // drop what touches a moonlet just matched; compact the rest in place (a pass
        // reads all its entries before any is written, and writes only below them)
        int kept = 0;
        for (int c0 = 0; c0 < nlive; c0 += U * T) {
            bool keep[U];
            int pv[U];
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int q = c0 + u * T + tid;
                keep[u] = false;
                pv[u] = 0;
                if (q < nlive) {
                    pv[u] = live[q];
                    if (flag[pv[u]] == 1) {
                        const int64_t k = keys[pv[u]];
                        if (mmatch[pair_i(k)] || mmatch[pair_j(k)]) flag[pv[u]] = 0;
                        else keep[u] = true;
                    }
                }
            }
            int cnt = 0;
#pragma unroll
            for (int u = 0; u < U; u++) cnt += keep[u] ? 1 : 0;
            int tot;
            int o = kept + block_int_prefix(cnt, wsum, &tot);
#pragma unroll
            for (int u = 0; u < U; u++)
                if (keep[u]) live[o++] = pv[u];
            kept += tot;
        }
        nlive = kept;
        __syncthreads();
    }
    // the resolved pairs, in (i, j) order, as (step, i, j) after the earlier steps';
    // a thread takes U consecutive pairs per pass
    const int64_t base = *cursor;
    int64_t run = 0;
    for (int c0 = 0; c0 < np; c0 += U * T) {
        bool acc[U];
        int cnt = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int p = c0 + U * tid + u;
            acc[u] = p < np && flag[p] == 2;
            cnt += acc[u] ? 1 : 0;
        }
        int tot;
        int64_t o = base + run + block_int_prefix(cnt, wsum, &tot);
#pragma unroll
        for (int u = 0; u < U; u++)
            if (acc[u]) {
                const int p = c0 + U * tid + u;
                if (o < cap) {
                    pairs[3 * o] = step;
                    pairs[3 * o + 1] = keys[p] >> 32;
                    pairs[3 * o + 2] = keys[p] & 0xffffffffll;
                }
                o++;
            }
        run += tot;
    }
    if (tid == 0) {
        *n_pairs_dev = run;
        if (base + run > cap) {
            atomicOr(&st->status, (int32_t)ST_CAP_PAIRS);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)(base + run));
        }
        *cursor = base + run;
    }
}

// Impulses of the resolved pairs (disjoint moonlets: 1 = i, 2 = j), over the whole GPU.
__global__ void __launch_bounds__(256)
k_resolve_apply(const DevState *__restrict__ st, const int64_t *__restrict__ keys,
                int64_t pair_cap, const int32_t *__restrict__ flag,
                const double *__restrict__ dtc, double *__restrict__ x,
                double *__restrict__ y, double *__restrict__ z, double *__restrict__ vx,
                double *__restrict__ vy, double *__restrict__ vz, const double *__restrict__ m,
                const double *__restrict__ R, double f) {
    const int np = resolve_count(st, pair_cap);
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < np; p += gridDim.x * blockDim.x) {
        if (flag[p] != 2) continue;
        const int64_t k = keys[p];
        const int i = pair_i(k), j = pair_j(k);
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
}

hipError_t launch_resolve(const Workspace &ws, double *x, double *y, double *z, double *vx,
                          double *vy, double *vz, const double *m, const double *R, double dt,
                          double f, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev, int step,
                          int64_t *cursor, const unsigned long long *tests_part, int n_part,
                          hipStream_t s) {
    const RankResolve RR = {x, y, z, vx, vy, vz, R, dt, ws.pair_dt, ws.pair_flag, ws.mmatch};
    k_rank_pairs<<<kRankGrid, kWave * kRankSplit, 0, s>>>(ws.st, ws.pairs_tmp, ws.pair_cap,
                                                          ws.pairs_alt, tests_part, n_part, RR);
    // the unsorted list is no longer needed: its buffer holds the live pair indices
    k_resolve<<<1, kResolveThreads, 0, s>>>(ws.st, ws.pairs_alt, ws.pair_cap, ws.pair_dt,
                                            ws.pair_flag, ws.mbest, ws.mmatch,
                                            (int32_t *)ws.pairs_tmp, pairs, cap, n_pairs_dev,
                                            step, cursor);
    k_resolve_apply<<<kResolveGrid, 256, 0, s>>>(ws.st, ws.pairs_alt, ws.pair_cap, ws.pair_flag,
                                                 ws.pair_dt, x, y, z, vx, vy, vz, m, R, f);
    return hipGetLastError();
}

hipError_t launch_collide_pairs(const Workspace &ws, int64_t n, double dt, bool boxes,
                                hipStream_t s) {
    (void)n;
    if (!boxes) k_collide_init<<<1, 64, 0, s>>>(ws.st);   // boxes: done by the box pass
    if (boxes) {
        k_collide<true><<<kCollideGrid, 64, 0, s>>>(ws.st, ws.cand, ws.p2p_cap, ws.c_first,
                                                    ws.c_count, ws.ccell, ws.cbox, ws.idx,
                                                    ws.pcol, ws.vcol, ws.ent_cell, dt,
                                                    ws.pairs_tmp, ws.pair_cap, ws.count_part);
        return hipGetLastError();
    }
    k_collide<false><<<kCollideGrid, 64, 0, s>>>(ws.st, ws.cand, ws.p2p_cap, ws.c_first,
                                                 ws.c_count, ws.ccell, ws.cbox, ws.idx, ws.pcol,
                                                 ws.vcol, ws.ent_cell, dt, ws.pairs_tmp,
                                                 ws.pair_cap, ws.count_part);
    return hipGetLastError();
}

hipError_t launch_emit_pairs(const Workspace &ws, int64_t *pairs, int64_t cap,
                             int64_t *n_pairs_dev, int triple, int step, int64_t *cursor,
                             const unsigned long long *tests_part, int n_part, hipStream_t s) {
    k_rank_pairs<<<kRankGrid, kWave * kRankSplit, 0, s>>>(ws.st, ws.pairs_tmp, ws.pair_cap,
                                                          ws.pairs_alt, tests_part, n_part,
                                                          RankResolve{});
    k_emit_pairs<<<256, 256, 0, s>>>(ws.st, ws.pairs_alt, ws.pair_cap, pairs, cap, n_pairs_dev,
                                     triple, step, cursor);
    k_pairs_done<<<1, 64, 0, s>>>(ws.st, n_pairs_dev, cap, ws.pair_cap, triple, cursor);
    return hipGetLastError();
}

}  // namespace ncorp

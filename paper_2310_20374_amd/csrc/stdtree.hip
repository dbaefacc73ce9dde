// Standard tree code (Alg. 1, Sect. 3.4.4) on the flat octree of the falcON path.
//
// Each wave takes 64 consecutive moonlets in tree (Hilbert) order and walks the
// tree once for all of them: a cell is visited while at least one lane still has
// to open it, and at every cell it reaches each lane takes the decision of Alg. 1
// for its own moonlet:
//   N_B < N_cb,pre                      -> direct sum over B's moonlets
//   |x - s_B| >= r_crit,B, x != s_B     -> cell-moonlet term C^(1)(x - s_B)
//   N_B < N_cb,post or B is a leaf      -> direct sum over B's moonlets
//   otherwise                           -> open B (its children are visited)
// so every moonlet's sum holds exactly the terms of its own walk, in the same
// depth-first order (children in increasing index).  A cell whose moonlets all
// sit at x has r_crit = 0; it is not separated from a moonlet there, where the
// expansion would be singular.
//
// Pending cells sit on a per-wave stack in LDS together with the mask of the
// lanes that reach them; the cell record, the multipoles and the source moonlets
// of a visited cell are the same for every lane of the wave and are read once per
// visit.  Because nearby moonlets take nearly the same decisions, the union of 64
// walks is not much longer than one of them.
//
// C^(1) of a cell B at x (Sect. 3.4.2, cell-moonlet form):
//   a_i = sum_{n=0, n!=1}^{p-1} (-1)^n sum_{|b|=n} D_{e_i+b}(x - s_B) Mt_b(B),
// D_g = d^g (1/|R|), Mt_b = M_b / b!, the moments of the gravity climb; the
// orders 0 and 2..p-1 are exactly the moments the climb keeps.
#include "contact.h"
#include "expansion.h"

namespace ncorp {
namespace {

constexpr int kStdBlock = 256;
constexpr int kStdWaves = kStdBlock / kWave;
// A visit pops one cell and pushes at most 8 children, so the stack holds at most
// 7 pending siblings for each level of the current path plus the 8 just pushed.
constexpr int kStdStack = 8 * kMaxDepth + 16;

__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// direct sum of the moonlets j in [b, e) on the moonlet at (x, y, z); a source at
// the same position (the moonlet itself) is skipped
__device__ __forceinline__ void direct_sum(const double *__restrict__ xs,
                                           const double *__restrict__ ys,
                                           const double *__restrict__ zs,
                                           const double *__restrict__ mus, int b, int e, double x,
                                           double y, double z, double &a0, double &a1,
                                           double &a2) {
    for (int j = b; j < e; j++) {
        const double dx = xs[j] - x, dy = ys[j] - y, dz = zs[j] - z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 == 0.0) continue;
        const double r = sqrt(r2);
        const double f = mus[j] / (r2 * r);      // one division per pair
        a0 += f * dx;
        a1 += f * dy;
        a2 += f * dz;
    }
}

template <int P>
__global__ __launch_bounds__(kStdBlock) void k_std_tree(
    DevState *st, const WCell *__restrict__ wg, const double *__restrict__ mult,
    const double *__restrict__ xs, const double *__restrict__ ys, const double *__restrict__ zs,
    const double *__restrict__ mus, const uint32_t *__restrict__ idx,
    const uint16_t *__restrict__ seg, const int32_t *__restrict__ disk_root, int64_t n,
    int ncb_pre, int ncb_post, double *__restrict__ ax, double *__restrict__ ay,
    double *__restrict__ az) {
    constexpr int NM = n_mult(P), ND = off_order(P + 1);
    __shared__ int32_t s_cell[kStdWaves][kStdStack];
    __shared__ uint64_t s_mask[kStdWaves][kStdStack];
    if (st->status & kSkipMask) return;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t k = ((int64_t)blockIdx.x * kStdWaves + w) * kWave + lane;
    const bool live = k < n;
    double x = 0.0, y = 0.0, z = 0.0;
    int root = 0;
    if (live) {
        x = xs[k]; y = ys[k]; z = zs[k];
        root = seg ? disk_root[seg[k]] : 0;
    }
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    bool overflow = false;
    // a wave can straddle disks of a batched call: one walk per distinct root
    uint64_t todo = __ballot(live);
    while (todo && !overflow) {
        const int r = __builtin_amdgcn_readlane(root, (int)__builtin_ctzll(todo));
        const uint64_t rm = __ballot(live && root == r);
        todo &= ~rm;
        if (lane == 0) { s_cell[w][0] = r; s_mask[w][0] = rm; }
        int sp = 1;
        while (sp > 0) {
            wave_sync();
            sp--;
            const int c = uniform_i32(s_cell[w][sp]);
            const uint64_t m = uniform_u64(s_mask[w][sp]);
            const WCell cw = wg[c];
            int action = 0;
            double dx = 0.0, dy = 0.0, dz = 0.0;
            if ((m >> lane) & 1) {
                dx = x - cw.x; dy = y - cw.y; dz = z - cw.z;
                const double d = sqrt(dx * dx + dy * dy + dz * dz);
                if (cw.count < ncb_pre) action = 1;
                else if (d >= cw.rcrit && d > 0.0) action = 2;
                else if (cw.count < ncb_post || cw.nchild == 0) action = 1;
                else action = 3;
            }
            const uint64_t open = __ballot(action == 3);
            if (open) {
                if (sp + cw.nchild > kStdStack) { overflow = true; break; }
                if (lane == 0)
                    for (int i = 0; i < cw.nchild; i++) {
                        s_cell[w][sp + i] = cw.child + cw.nchild - 1 - i;
                        s_mask[w][sp + i] = open;
                    }
                sp += cw.nchild;
            }
            if (__ballot(action == 2)) {
                if (action == 2) {
                    double D[ND];
                    green_derivs<P, double>(dx, dy, dz, rsqrt_t<double>(dx * dx + dy * dy + dz * dz),
                                            D);
                    double acc[3] = {0.0, 0.0, 0.0};
                    m2l_contract<P, 1, 1, double>(D, mult + (int64_t)c * NM, acc);
                    a0 += acc[0]; a1 += acc[1]; a2 += acc[2];
                }
            }
            if (__ballot(action == 1)) {
                if (action == 1)
                    direct_sum(xs, ys, zs, mus, cw.first, cw.first + cw.count, x, y, z, a0, a1, a2);
            }
        }
    }
    if (overflow) {
        if (lane == 0) atomicOr(&st->status, (int32_t)ST_BAD_ITEM);
        return;
    }
    if (live) {
        const uint32_t i = idx[k];
        ax[i] = a0; ay[i] = a1; az[i] = a2;
    }
}

// Collision search by the standard tree code (Alg. 1 in its collision form): the same
// per-moonlet walk over the collision climb's cells (centre s_B, radius r_crit,B that
// holds every moonlet of B with its reach R + dt |v|).  A cell is separated from
// moonlet a when |x_a - s_B| >= (R_a + dt |v_a| + r_crit,B)(1 + 1e-9): no moonlet of B
// can then meet a within the step, and the walk does nothing; the margin dwarfs the
// rounding of either radius.  Brute-forced cells test every (a, j) with input index
// i_a < i_j exactly (Eqs. 1-2); since no colliding partner of a is ever in a
// separated cell, a's own walk finds all pairs (a, j) with i_a < i_j, so every
// colliding pair is found exactly once.
__global__ __launch_bounds__(kStdBlock) void k_std_collide(
    DevState *st, const WCell *__restrict__ wc, const double4 *__restrict__ pcol,
    const double *__restrict__ xs, const double *__restrict__ ys, const double *__restrict__ zs,
    const double *__restrict__ vxs, const double *__restrict__ vys, const double *__restrict__ vzs,
    const double *__restrict__ rads, const uint32_t *__restrict__ idx,
    const uint16_t *__restrict__ seg, const int32_t *__restrict__ disk_root, int64_t n,
    int ncb_pre, int ncb_post, double dt, int64_t *out, int64_t cap,
    unsigned long long *tests_part) {
    __shared__ int32_t s_cell[kStdWaves][kStdStack];
    __shared__ uint64_t s_mask[kStdWaves][kStdStack];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const int64_t wave = (int64_t)blockIdx.x * kStdWaves + w;
    if (st->status & kSkipMask) {
        if (lane == 0) tests_part[wave] = 0;
        return;
    }
    const int64_t k = wave * kWave + lane;
    const bool live = k < n;
    double4 me = make_double4(0.0, 0.0, 0.0, 0.0);
    double vx = 0.0, vy = 0.0, vz = 0.0, R = 0.0;
    uint32_t id = 0;
    int root = 0;
    if (live) {
        me = pcol[k];
        vx = vxs[k]; vy = vys[k]; vz = vzs[k]; R = rads[k];
        id = idx[k];
        root = seg ? disk_root[seg[k]] : 0;
    }
    unsigned long long tests = 0;
    bool overflow = false;
    uint64_t todo = __ballot(live);
    while (todo && !overflow) {
        const int r = __builtin_amdgcn_readlane(root, (int)__builtin_ctzll(todo));
        const uint64_t rm = __ballot(live && root == r);
        todo &= ~rm;
        if (lane == 0) { s_cell[w][0] = r; s_mask[w][0] = rm; }
        int sp = 1;
        while (sp > 0) {
            wave_sync();
            sp--;
            const int c = uniform_i32(s_cell[w][sp]);
            const uint64_t m = uniform_u64(s_mask[w][sp]);
            const WCell cw = wc[c];
            int action = 0;
            if ((m >> lane) & 1) {
                const double dx = me.x - cw.x, dy = me.y - cw.y, dz = me.z - cw.z;
                const double rs = (me.w + cw.rcrit) * (1.0 + 1e-9);
                if (cw.count < ncb_pre) action = 1;
                else if (dx * dx + dy * dy + dz * dz >= rs * rs) action = 0;
                else if (cw.count < ncb_post || cw.nchild == 0) action = 1;
                else action = 3;
            }
            const uint64_t open = __ballot(action == 3);
            if (open) {
                if (sp + cw.nchild > kStdStack) { overflow = true; break; }
                if (lane == 0)
                    for (int i = 0; i < cw.nchild; i++) {
                        s_cell[w][sp + i] = cw.child + cw.nchild - 1 - i;
                        s_mask[w][sp + i] = open;
                    }
                sp += cw.nchild;
            }
            if (__ballot(action == 1)) {
                if (action == 1) {
                    for (int j = cw.first; j < cw.first + cw.count; j++) {
                        const uint32_t jd = idx[j];
                        if (jd <= id) continue;
                        tests++;
                        if (pair_test(me.x, me.y, me.z, vx, vy, vz, R, xs[j], ys[j], zs[j],
                                      vxs[j], vys[j], vzs[j], rads[j], dt))
                            record(out, cap, (unsigned long long *)&st->npairs, id, jd);
                    }
                }
            }
        }
    }
    if (overflow && lane == 0) atomicOr(&st->status, (int32_t)ST_BAD_ITEM);
    for (int o = 32; o > 0; o >>= 1) tests += __shfl_xor(tests, o);
    if (lane == 0) tests_part[wave] = tests;
}

template <int P>
hipError_t launch_std_t(const Workspace &ws, int64_t n, int ncb_pre, int ncb_post, double *ax,
                        double *ay, double *az, hipStream_t s) {
    const int64_t blocks = (n + kStdBlock - 1) / kStdBlock;
    k_std_tree<P><<<(unsigned)blocks, kStdBlock, 0, s>>>(
        ws.st, ws.wg, ws.mult, ws.xs, ws.ys, ws.zs, ws.mus, ws.idx,
        ws.ndisks > 1 ? ws.seg : nullptr, ws.disk_root, n, ncb_pre, ncb_post, ax, ay, az);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_standard_tree_collide(const Workspace &ws, int64_t n, int ncb_pre,
                                        int ncb_post, double dt, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + kStdBlock - 1) / kStdBlock;
    k_std_collide<<<(unsigned)blocks, kStdBlock, 0, s>>>(
        ws.st, ws.wc, ws.pcol, ws.xs, ws.ys, ws.zs, ws.vxs, ws.vys, ws.vzs, ws.rads, ws.idx,
        ws.ndisks > 1 ? ws.seg : nullptr, ws.disk_root, n, ncb_pre, ncb_post, dt, ws.pairs_tmp,
        ws.pair_cap, ws.count_part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_u64(ws.count_part, blocks * kStdWaves,
                          (unsigned long long *)&ws.st->col_tests, true, s);
}

hipError_t launch_standard_tree(const Workspace &ws, int64_t n, int p, int ncb_pre, int ncb_post,
                                double *ax, double *ay, double *az, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (p) {
        case 1: return launch_std_t<1>(ws, n, ncb_pre, ncb_post, ax, ay, az, s);
        case 2: return launch_std_t<2>(ws, n, ncb_pre, ncb_post, ax, ay, az, s);
        case 3: return launch_std_t<3>(ws, n, ncb_pre, ncb_post, ax, ay, az, s);
        case 4: return launch_std_t<4>(ws, n, ncb_pre, ncb_post, ax, ay, az, s);
        case 5: return launch_std_t<5>(ws, n, ncb_pre, ncb_post, ax, ay, az, s);
        case 6: return launch_std_t<6>(ws, n, ncb_pre, ncb_post, ax, ay, az, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ncorp

// Tree climbs (Sect. 3.4.2).  One wave per leaf computes the leaf, then walks up:
// each finished cell bumps its parent's arrival counter and the wave that arrives
// last computes the parent from its (complete) children.  No wave ever waits, so
// the pass is a single launch with no level loop.
//
// Gravity: centre of mass (Eq. 10), r_max (Eq. 11) clamped to the farthest corner
// of the cell's cube, scaled multipole moments Mt_a = M_a / a! (Eq. 20 at leaves,
// binomial shift of App. C above), then theta(M) and r_crit = r_max/theta (Eq. 12)
// once the root mass is known.  Collisions: centroid (Eq. 7), r_max (Eq. 8) and
// r_crit (Eq. 9) with r_crit - r_max = R + dt |v| for a moonlet.
//
// Operation order of the centres, radii and angles is fixed (children or moonlets
// in tree order, no contraction) so they are reproducible bit for bit.
#include "ncorp_internal.h"
#include "rcrit.h"

namespace ncorp {

__device__ __forceinline__ double dist3(double ax, double ay, double az, double bx, double by,
                                        double bz) {
    double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

__device__ __forceinline__ uint32_t quantize_c(double x, double L, double scale) {
    double t = (x + L) * scale;
    if (!(t >= 0.0)) return 0u;
    if (t >= 2097152.0) return 2097151u;
    uint32_t q = (uint32_t)floor(t);
    return q > 2097151u ? 2097151u : q;
}

// distance from (sx, sy, sz) to the farthest corner of the cell's cube; the cube
// follows from any moonlet of the cell (here its first) and the cell's level
__device__ double far_corner(double sx, double sy, double sz, double px, double py, double pz,
                             int level, double L) {
    double scale = 1048576.0 / L;
    int sh = kMaxDepth - level;
    double cx = (double)(quantize_c(px, L, scale) >> sh);
    double cy = (double)(quantize_c(py, L, scale) >> sh);
    double cz = (double)(quantize_c(pz, L, scale) >> sh);
    double hw = ldexp(L, -level);
    double side = ldexp(1.0, level);
    double ex = hw * (2.0 * cx + 1.0 - side);
    double ey = hw * (2.0 * cy + 1.0 - side);
    double ez = hw * (2.0 * cz + 1.0 - side);
    double dx = fabs(sx - ex) + hw, dy = fabs(sy - ey) + hw, dz = fabs(sz - ez) + hw;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// moonlets whose scaled powers are staged in LDS at a time (a leaf holds at most
// s of them, typically a few dozen)
constexpr int kPowChunk = 32;

// Leaves of the climbs in XCD slices: the leaves, in tree order, are cut into 8
// contiguous slices and the waves of XCD x (workgroups b with b mod 8 = x) take the
// leaves of slice x in order: the first of each wave by its position, later ones
// one at a time from a counter of that slice.  Siblings
// and most of their ancestors' chains then stay on one XCD and every XCD gets the
// same number of leaves (with leaves dealt round robin, an XCD that falls behind
// arrives last more often, inherits more of the upward chains and falls further
// behind).  The waves are persistent, as many as fit on the chip at once, so no
// leaf waits for a workgroup launch.

template <int KERNEL_ID>
static int climb_grid(const void *kernel, int64_t leaf_cap) {
    static int cached[64] = {};                     // per device, for this kernel
    int dev = 0;
    (void)hipGetDevice(&dev);
    int g = dev >= 0 && dev < 64 ? cached[dev] : 0;
    if (g == 0) {
        int per_cu = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kWave, 0) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            per_cu < 1 || ncu < 1) {
            (void)hipGetLastError();
            per_cu = 16;
            ncu = 256;
        }
        g = per_cu * ncu / kXcds * kXcds;
        if (g < kXcds) g = kXcds;
        if (dev >= 0 && dev < 64) cached[dev] = g;
    }
    int64_t want = (leaf_cap + kXcds - 1) / kXcds * kXcds;
    if (want < kXcds) want = kXcds;
    return (int)(want < g ? want : g);
}

// next leaf index of this wave's slice after the first round (lane 0 takes it from
// the slice's counter; every lane reads it later)
__device__ __forceinline__ int take_leaf(int32_t *ctr) {
    int i = 0;
    if (threadIdx.x == 0) i = atomicAdd(ctr, 1) + (int)(gridDim.x / kXcds);
    return i;
}

// ---------------------------------------------------------------- wave helpers
// Cell results are handed from wave to wave inside one launch: they are written
// with agent-coherent stores and read back with agent-coherent loads, and a wave
// waits for its stores to complete before it bumps the parent's arrival counter.
// The arrival counter's returned value orders the parent's loads after it.  (A
// full device fence here would write back and invalidate the L2 at every cell.)
__device__ __forceinline__ void st_c(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_c(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// 1 if this wave is the last of the parent's children to arrive
__device__ __forceinline__ bool arrive_last(int32_t *counter, int nchild) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);                 // this wave's stores are complete
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    int old = 0;
    if (threadIdx.x == 0) old = atomicAdd(counter, 1);
    old = __builtin_amdgcn_readlane(old, 0);       // wave-uniform: a scalar branch
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return old == nchild - 1;
}

// M2M sums of lane j's shift terms over NQ children (children nch..NQ-1 of the
// staged tables are zeros): one partial sum per child, added in child order
template <int NQ, int NE, int NMS>
__device__ __forceinline__ double m2m_terms(const uint16_t *sterm, int t0, int t1,
                                            const double (*cm)[NMS], const double (*ue)[NE]) {
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; q++) acc[q] = 0.0;
    int w = sterm[t0];                  // sterm has one entry past the last term
    for (int t = t0; t < t1; t++) {
        const int wn = sterm[t + 1];
        const int src = w & 63, ex = w >> 6;
#pragma unroll
        for (int q = 0; q < NQ; q++) acc[q] += cm[q][src] * ue[q][ex];
        w = wn;
    }
    double s = acc[0];
#pragma unroll
    for (int q = 1; q < NQ; q++) s += acc[q];
    return s;
}

// value of lane k (k uniform)
__device__ __forceinline__ double rl(double v, int k) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return v;
}

// multi-index (a, b, c) of multipole slot j (0 <= j < n_mult(p))
__host__ __device__ constexpr void mult_index(int j, int &a, int &b, int &c) {
    if (j == 0) { a = b = c = 0; return; }
    const int s = j + 3;
    int n = 2;
    while (off_order(n + 1) <= s) n++;
    const int r = s - off_order(n);
    int k = 0;
    while (tri(k + 1) <= r) k++;
    c = r - tri(k);
    b = k - c;
    a = n - k;
}

// multi-index (a, b, c) of position s among all orders (inverse of sidx)
__host__ __device__ constexpr void sidx_inverse(int s, int &a, int &b, int &c) {
    int n = 0;
    while (off_order(n + 1) <= s) n++;
    const int r = s - off_order(n);
    int k = 0;
    while (tri(k + 1) <= r) k++;
    c = r - tri(k);
    b = k - c;
    a = n - k;
}

// Terms of the App. C shift Mt_a(s') = sum_{b <= a, |b| != 1} Mt_b(s) u^(a-b)/(a-b)!
// for every multipole slot: term t of slot j (first[j] <= t < first[j+1]) packs
// the source slot (6 bits) and the position of the exponent e = a - b among all
// multi-indices of order < p (sidx, 6 bits).
template <int P> struct ShiftTerms {
    static constexpr int NM = n_mult(P);
    static constexpr int count() {
        int t = 0;
        for (int j = 0; j < NM; j++) {
            int a = 0, b = 0, c = 0;
            mult_index(j, a, b, c);
            for (int a2 = 0; a2 <= a; a2++)
                for (int b2 = 0; b2 <= b; b2++)
                    for (int c2 = 0; c2 <= c; c2++)
                        if (a2 + b2 + c2 != 1) t++;
        }
        return t;
    }
    static constexpr int NT = count() > 0 ? count() : 1;
    uint16_t first[NM + 1];
    uint16_t term[NT];
    constexpr ShiftTerms() : first(), term() {
        int t = 0;
        for (int j = 0; j < NM; j++) {
            first[j] = (uint16_t)t;
            int a = 0, b = 0, c = 0;
            mult_index(j, a, b, c);
            for (int a2 = 0; a2 <= a; a2++)
                for (int b2 = 0; b2 <= b; b2++)
                    for (int c2 = 0; c2 <= c; c2++)
                        if (a2 + b2 + c2 != 1)
                            term[t++] = (uint16_t)(midx(a2, b2, c2) |
                                                   (sidx(a - a2, b - b2, c - c2) << 6));
        }
        first[NM] = (uint16_t)t;
    }
};
template <int P> __constant__ ShiftTerms<P> kShift = ShiftTerms<P>();

// Gravity climb.  One wave per cell.  Centre of mass: the sums over moonlets
// (leaves) or children (internal cells) are formed in a fixed sequential order, so
// they are reproducible bit for bit (at a leaf lane j < 4 forms the sum of
// mu * (1, x, y, z)_j, mu * 1 being mu exactly); r_max is an exact wave maximum.
// Moments: lane j owns multipole slot j.  At a leaf each lane first stages its
// moonlet's scaled powers u^k/k! in LDS, then lane j sums mu u^a/a! over the
// moonlets in order (Eq. 20).  At an internal cell the children's moments and the
// products u^e/e! of their offsets' scaled powers (one exponent e per lane, every
// e of order < p) are staged in LDS, and lane j sums its slot's shift terms for
// each child.  Between levels a wave issues the parent's tree links before it
// waits for its own stores, and every load of the parent's inputs at once after the
// arrival counter; the cell index and the child count are wave-uniform throughout.
template <int P>
__global__ void __launch_bounds__(kWave)
k_gravity_climb(const DevState *__restrict__ st, const double *__restrict__ xs,
                const double *__restrict__ ys, const double *__restrict__ zs,
                const double *__restrict__ mus, const int32_t *__restrict__ ent_cell,
                const int32_t *__restrict__ c_level, const int32_t *__restrict__ c_first,
                const int32_t *__restrict__ c_count, const int32_t *__restrict__ c_child,
                const int32_t *__restrict__ c_nchild, const int32_t *__restrict__ c_parent,
                int32_t *c_arrive, int32_t *climb_next, double4 *gcell, double *c_mass,
                double *c_rmax,
                double *mult, float *mult32, const uint16_t *__restrict__ seg,
                const double *__restrict__ disk_L) {
    constexpr int NM = n_mult(P);
    constexpr int NP = P > 1 ? P : 1;               // powers 0..P-1
    constexpr int NMS = NM > 0 ? NM : 1;
    constexpr int NE = off_order(P) > 0 ? off_order(P) : 1;   // exponents of order < P
    static_assert(NE <= kWave && NM <= kWave, "one lane per exponent and per slot");
    // LDS, reused between the phases: the leaf's centre of mass stages (1, x, y, z)
    // and the masses of 64 moonlets, its P2M the scaled powers and masses of
    // kPowChunk moonlets; a parent (M2M) the powers of its <= 8 children's offsets,
    // then their products U[child][e] and the children's moments
    constexpr int kComDbl = kWave * 5;
    constexpr int kLeafDbl = kPowChunk * 3 * NP + kPowChunk;
    constexpr int kParentDbl = 8 * NE + 8 * NMS;
    constexpr int kA = kComDbl > kLeafDbl ? kComDbl : kLeafDbl;
    constexpr int kB = kParentDbl > 8 * 3 * NP ? kParentDbl : 8 * 3 * NP;
    __shared__ double buf[kA > kB ? kA : kB];
    double (*sq)[4] = reinterpret_cast<double (*)[4]>(buf);           // leaf COM: (1, x, y, z)
    double *sqm = buf + kWave * 4;                                    // leaf COM: masses
    double (*pw)[3][NP] = reinterpret_cast<double (*)[3][NP]>(buf);   // [moonlet/child][axis][k]
    double *smu = buf + kPowChunk * 3 * NP;                           // leaf P2M: masses
    double (*ue)[NE] = reinterpret_cast<double (*)[NE]>(buf);         // parent: U[child][e]
    double (*cm)[NMS] = reinterpret_cast<double (*)[NMS]>(buf + 8 * NE);  // parent: moments
    __shared__ uint16_t sterm[ShiftTerms<P>::NT + 1];   // shift terms (from constant memory)
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    const double L = st->L;
    const int lane = threadIdx.x;
    int ja = 0, jb = 0, jc = 0, t0 = 0, t1 = 0, ea = 0, eb = 0, ec = 0;
    if (lane < NM) {
        mult_index(lane, ja, jb, jc);
        t0 = kShift<P>.first[lane];
        t1 = kShift<P>.first[lane + 1];
    }
    if (lane < NE) sidx_inverse(lane, ea, eb, ec);
    for (int t = lane; t < ShiftTerms<P>::NT; t += kWave) sterm[t] = kShift<P>.term[t];
    if (lane == 0) sterm[ShiftTerms<P>::NT] = 0;
    __syncthreads();
    const int per = (K + kXcds - 1) / kXcds;       // leaves per XCD slice
    const int xcd = (int)blockIdx.x % kXcds;
    int32_t *ctr = climb_next + xcd * kCtrStride;
    int nxt = (int)blockIdx.x / kXcds;             // first round: one leaf per wave, no counter
    for (;;) {
        const int i = __builtin_amdgcn_readlane(nxt, 0);
        const int e = xcd * per + i;
        if (i >= per || e >= K) break;
        nxt = take_leaf(ctr);                       // the next one, in flight meanwhile
        int c = __builtin_amdgcn_readfirstlane(ent_cell[e]);
        int par = __builtin_amdgcn_readfirstlane(c_parent[c]);
        // ---- leaf: moonlets f .. f+cnt-1
        {
            const int f = __builtin_amdgcn_readfirstlane(c_first[c]);
            const int cnt = __builtin_amdgcn_readfirstlane(c_count[c]);
            double acc4 = 0.0;
            for (int c0 = 0; c0 < cnt; c0 += kWave) {
                const bool in = c0 + lane < cnt;
                const int k = f + c0 + (in ? lane : 0);
                const double mu = mus[k], x = xs[k], y = ys[k], z = zs[k];
                __syncthreads();
                sq[lane][0] = 1.0; sq[lane][1] = x; sq[lane][2] = y; sq[lane][3] = z;
                sqm[lane] = mu;
                __syncthreads();
                const int nk = cnt - c0 < kWave ? cnt - c0 : kWave;
                if (lane < 4) {
#pragma unroll 8
                    for (int q = 0; q < nk; q++) acc4 += sqm[q] * sq[q][lane];
                }
            }
            const double M = rl(acc4, 0);
            const double sx = rl(acc4, 1) / M, sy = rl(acc4, 2) / M, sz = rl(acc4, 3) / M;
            double rm = 0.0, acc = 0.0;
            for (int c0 = 0; c0 < cnt; c0 += kPowChunk) {
                const bool in = lane < kPowChunk && c0 + lane < cnt;
                const int k = f + c0 + (in ? lane : 0);
                const double mu = mus[k], x = xs[k], y = ys[k], z = zs[k];
                if (in) {
                    const double d = 0.0 + dist3(x, y, z, sx, sy, sz);
                    if (d > rm) rm = d;
                }
                if (NM > 0) {
                    const int nk = cnt - c0 < kPowChunk ? cnt - c0 : kPowChunk;
                    __syncthreads();
                    if (lane < kPowChunk) {
                        const double ux = x - sx, uy = y - sy, uz = z - sz;
                        double tx = 1.0, ty = 1.0, tz = 1.0;
                        pw[lane][0][0] = 1.0; pw[lane][1][0] = 1.0; pw[lane][2][0] = 1.0;
#pragma unroll
                        for (int i = 1; i < NP; i++) {
                            tx = tx * ux * (1.0 / (double)i);
                            ty = ty * uy * (1.0 / (double)i);
                            tz = tz * uz * (1.0 / (double)i);
                            pw[lane][0][i] = tx; pw[lane][1][i] = ty; pw[lane][2][i] = tz;
                        }
                        smu[lane] = mu;
                    }
                    __syncthreads();
                    if (lane < NM) {
#pragma unroll 4
                        for (int q = 0; q < nk; q++)
                            acc += smu[q] * (pw[q][0][ja] * pw[q][1][jb] * pw[q][2][jc]);
                    }
                }
            }
            rm = wave_max(rm);
            const double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c],
                                         seg ? disk_L[seg[f]] : L);
            if (fc < rm) rm = fc;
            if (lane == 0) {
                st_c(&gcell[c].x, sx); st_c(&gcell[c].y, sy); st_c(&gcell[c].z, sz);
                st_c(&gcell[c].w, 0.0);
                st_c(&c_mass[c], M);
                st_c(&c_rmax[c], rm);
            }
            if (lane < NM) {
                st_c(&mult[(int64_t)c * NM + lane], acc);
                mult32[(int64_t)c * NM + lane] = (float)acc;
            }
        }
        // ---- walk up while this wave is the last child to arrive
        for (int up = 0; up < kMaxDepth && par >= 0; up++) {   // one step per level
            // the parent's tree links are fixed during the climb: plain loads, in flight
            // while this wave's stores complete
            const int a0 = __builtin_amdgcn_readfirstlane(c_child[par]);
            const int nch = __builtin_amdgcn_readfirstlane(c_nchild[par]);
            const int f = __builtin_amdgcn_readfirstlane(c_first[par]);
            const int lev = __builtin_amdgcn_readfirstlane(c_level[par]);
            const int gpar = __builtin_amdgcn_readfirstlane(c_parent[par]);
            if (!arrive_last(&c_arrive[par], nch)) break;
            c = par;
            par = gpar;
            const bool in = lane < nch;
            const int a = a0 + (in ? lane : 0);
            const double ma_ = ld_c(&c_mass[a]);
            const double gx = ld_c(&gcell[a].x), gy = ld_c(&gcell[a].y), gz = ld_c(&gcell[a].z);
            const double ra = ld_c(&c_rmax[a]);
            double mq[8];
#pragma unroll
            for (int q = 0; q < 8; q++)
                mq[q] = (NM > 0 && q < nch && lane < NM)
                            ? ld_c(&mult[(int64_t)(a0 + q) * NM + lane]) : 0.0;
            const double px = xs[f], py = ys[f], pz = zs[f];
            const double Lc = seg ? disk_L[seg[f]] : L;
            double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int q = 0; q < nch; q++) M += rl(ma_, q);
            for (int q = 0; q < nch; q++) {
                const double m = rl(ma_, q);
                sx += m * rl(gx, q);
                sy += m * rl(gy, q);
                sz += m * rl(gz, q);
            }
            sx = sx / M; sy = sy / M; sz = sz / M;
            double rm = 0.0;
            if (in) {
                const double d = ra + dist3(gx, gy, gz, sx, sy, sz);
                if (d > rm) rm = d;
            }
            rm = wave_max(rm);
            const double fc = far_corner(sx, sy, sz, px, py, pz, lev, Lc);
            if (fc < rm) rm = fc;
            if (lane == 0) {
                st_c(&gcell[c].x, sx); st_c(&gcell[c].y, sy); st_c(&gcell[c].z, sz);
                st_c(&gcell[c].w, 0.0);
                st_c(&c_mass[c], M);
                st_c(&c_rmax[c], rm);
            }
            if (NM > 0) {
                __syncthreads();
                // u^k/k! of each child's offset (lane = child)
                if (in) {
                    const double ux = gx - sx, uy = gy - sy, uz = gz - sz;
                    double tx = 1.0, ty = 1.0, tz = 1.0;
                    pw[lane][0][0] = 1.0; pw[lane][1][0] = 1.0; pw[lane][2][0] = 1.0;
#pragma unroll
                    for (int i = 1; i < NP; i++) {
                        tx = tx * ux * (1.0 / (double)i);
                        ty = ty * uy * (1.0 / (double)i);
                        tz = tz * uz * (1.0 / (double)i);
                        pw[lane][0][i] = tx; pw[lane][1][i] = ty; pw[lane][2][i] = tz;
                    }
                }
                __syncthreads();
                // U[child][e] = u^e/e!, lane = e
                double u[8];
#pragma unroll
                for (int q = 0; q < 8; q++)
                    u[q] = (q < nch && lane < NE)
                               ? pw[q][0][ea] * pw[q][1][eb] * pw[q][2][ec] : 0.0;
                __syncthreads();
                const int nq = nch <= 4 ? 4 : 8;   // staged children, zeros past nch
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    if (q < nq && lane < NE) ue[q][lane] = u[q];
                    if (q < nq && lane < NM) cm[q][lane] = mq[q];
                }
                __syncthreads();
                if (lane < NM) {
                    const double acc = nq == 4 ? m2m_terms<4, NE, NMS>(sterm, t0, t1, cm, ue)
                                               : m2m_terms<8, NE, NMS>(sterm, t0, t1, cm, ue);
                    st_c(&mult[(int64_t)c * NM + lane], acc);
                    mult32[(int64_t)c * NM + lane] = (float)acc;
                }
            }
        }
    }
}

__global__ void k_rcrit(const DevState *__restrict__ st, const RcritArgs R) {
    const int nc = st->ncells;
    if (nc <= 0 || (st->status & kSkipMask)) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
        rcrit_cell(R, c);
}

__global__ void k_pack_collision(const DevState *__restrict__ st, const double4 *__restrict__ ccell,
                                 const int32_t *__restrict__ c_count,
                                 const int32_t *__restrict__ c_child,
                                 const int32_t *__restrict__ c_nchild, WCell *__restrict__ wc,
                                 const int32_t *__restrict__ c_entry,
                                 const int32_t *__restrict__ c_nent,
                                 const int32_t *__restrict__ c_first) {
    const int nc = st->ncells;
    if (st->status & kSkipMask) return;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
        const double4 g = ccell[c];
        WCell w;
        w.x = g.x; w.y = g.y; w.z = g.z; w.rcrit = g.w;
        w.count = c_count[c]; w.child = c_child[c]; w.nchild = c_nchild[c];
        w.entry = c_entry[c]; w.nent = c_nent[c]; w.first = c_first[c]; w.pad[0] = w.pad[1] = 0;
        wc[c] = w;
    }
}

__global__ void k_arrive_reset(const DevState *__restrict__ st, int32_t *c_arrive,
                               int32_t *climb_next) {
    const int nc = st->ncells;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x)
        c_arrive[c] = 0;
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < kXcds * kCtrStride; t += blockDim.x) climb_next[t] = 0;
}

static int cell_grid(int64_t cap, int block) {
    int64_t g = (cap + block - 1) / block;
    return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

template <int P>
static void launch_gc(const Workspace &ws, hipStream_t s) {
    const int g = climb_grid<P>((const void *)k_gravity_climb<P>, ws.leaf_cap);
    k_gravity_climb<P><<<g, kWave, 0, s>>>(ws.st, ws.xs, ws.ys, ws.zs, ws.mus, ws.ent_cell,
                                         ws.c_level, ws.c_first, ws.c_count, ws.c_child,
                                         ws.c_nchild, ws.c_parent, ws.c_arrive, ws.climb_next,
                                         ws.gcell,
                                         ws.c_mass, ws.c_rmax, ws.mult, ws.mult32,
                                         ws.ndisks > 1 ? ws.seg : nullptr, ws.disk_L);
}

hipError_t launch_gravity_climb(const Workspace &ws, int64_t n, const ncorp_params &prm,
                                hipStream_t s, bool reset, bool rcrit) {
    (void)n;
    if (reset)
        k_arrive_reset<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.c_arrive,
                                                                   ws.climb_next);
    switch (prm.p) {
        case 0: launch_gc<0>(ws, s); break;
        case 1: launch_gc<1>(ws, s); break;
        case 2: launch_gc<2>(ws, s); break;
        case 3: launch_gc<3>(ws, s); break;
        case 4: launch_gc<4>(ws, s); break;
        case 5: launch_gc<5>(ws, s); break;
        default: launch_gc<6>(ws, s); break;
    }
    if (rcrit)
        k_rcrit<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, rcrit_args(ws, prm));
    return hipGetLastError();
}

// ------------------------------------------------------------------ collisions
// Same scheme: one wave per cell, centroid summed sequentially (bit-reproducible),
// r_max and the largest R + dt |v| as exact wave maxima.
__global__ void __launch_bounds__(kWave)
k_collision_climb(const DevState *__restrict__ st, const double *__restrict__ xs,
                  const double *__restrict__ ys, const double *__restrict__ zs,
                  const double *__restrict__ vxs, const double *__restrict__ vys,
                  const double *__restrict__ vzs, const double *__restrict__ rads, double dt,
                  const int32_t *__restrict__ ent_cell, const int32_t *__restrict__ c_level,
                  const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
                  const int32_t *__restrict__ c_child, const int32_t *__restrict__ c_nchild,
                  const int32_t *__restrict__ c_parent, int32_t *c_arrive,
                  int32_t *climb_next, double4 *ccell,
                  double *c_crmax,
                  const uint16_t *__restrict__ seg, const double *__restrict__ disk_L,
                  double4 *__restrict__ pcol) {
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    const double L = st->L;
    const int lane = threadIdx.x;
    const int per = (K + kXcds - 1) / kXcds;       // leaves per XCD slice
    const int xcd = (int)blockIdx.x % kXcds;
    int32_t *ctr = climb_next + xcd * kCtrStride;
    int nxt = (int)blockIdx.x / kXcds;             // first round: one leaf per wave, no counter
    for (;;) {
        const int i = __builtin_amdgcn_readlane(nxt, 0);
        const int e = xcd * per + i;
        if (i >= per || e >= K) break;
        nxt = take_leaf(ctr);                       // the next one, in flight meanwhile
        int c = ent_cell[e];
        {
            const int f = c_first[c], cnt = c_count[c];
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int c0 = 0; c0 < cnt; c0 += kWave) {
                const int k = f + c0 + (c0 + lane < cnt ? lane : 0);
                const double x = xs[k], y = ys[k], z = zs[k];
                const int nk = cnt - c0 < kWave ? cnt - c0 : kWave;
                for (int q = 0; q < nk; q++) {
                    sx += rl(x, q);
                    sy += rl(y, q);
                    sz += rl(z, q);
                }
            }
            const double NA = (double)cnt;
            sx = sx / NA; sy = sy / NA; sz = sz / NA;
            double rm = 0.0, ex = 0.0;
            for (int c0 = 0; c0 < cnt; c0 += kWave) {
                if (c0 + lane < cnt) {
                    const int k = f + c0 + lane;
                    const double d = 0.0 + dist3(xs[k], ys[k], zs[k], sx, sy, sz);
                    if (d > rm) rm = d;
                    const double v = sqrt(vxs[k] * vxs[k] + vys[k] * vys[k] + vzs[k] * vzs[k]);
                    const double ee = (rads[k] + dt * v) - 0.0;
                    if (ee > ex) ex = ee;
                    pcol[k] = make_double4(xs[k], ys[k], zs[k], ee);
                }
            }
            rm = wave_max(rm);
            ex = wave_max(ex);
            const double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c],
                                         seg ? disk_L[seg[f]] : L);
            if (fc < rm) rm = fc;
            if (lane == 0) {
                st_c(&ccell[c].x, sx); st_c(&ccell[c].y, sy); st_c(&ccell[c].z, sz);
                st_c(&ccell[c].w, rm + ex);
                st_c(&c_crmax[c], rm);
            }
        }
        for (int up = 0; up < kMaxDepth; up++) {      // at most one step per level
            const int par = c_parent[c];
            if (par < 0) break;
            if (!arrive_last(&c_arrive[par], c_nchild[par])) break;
            c = par;
            const int a0 = c_child[c], nch = c_nchild[c];
            const bool in = lane < nch;
            const int a = a0 + (in ? lane : 0);
            const double na = (double)c_count[a];
            const double4 ca = make_double4(ld_c(&ccell[a].x), ld_c(&ccell[a].y),
                                            ld_c(&ccell[a].z), ld_c(&ccell[a].w));
            const double rma = ld_c(&c_crmax[a]);
            const double NA = (double)c_count[c];
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int q = 0; q < nch; q++) {
                const double w = rl(na, q);
                sx += w * rl(ca.x, q);
                sy += w * rl(ca.y, q);
                sz += w * rl(ca.z, q);
            }
            sx = sx / NA; sy = sy / NA; sz = sz / NA;
            double rm = 0.0, ex = 0.0;
            if (in) {
                const double d = rma + dist3(ca.x, ca.y, ca.z, sx, sy, sz);
                if (d > rm) rm = d;
                const double ee = ca.w - rma;
                if (ee > ex) ex = ee;
            }
            rm = wave_max(rm);
            ex = wave_max(ex);
            const int f = c_first[c];
            const double fc = far_corner(sx, sy, sz, xs[f], ys[f], zs[f], c_level[c],
                                         seg ? disk_L[seg[f]] : L);
            if (fc < rm) rm = fc;
            if (lane == 0) {
                st_c(&ccell[c].x, sx); st_c(&ccell[c].y, sy); st_c(&ccell[c].z, sz);
                st_c(&ccell[c].w, rm + ex);
                st_c(&c_crmax[c], rm);
            }
        }
    }
}

hipError_t launch_collision_climb(const Workspace &ws, int64_t n, double dt, hipStream_t s,
                                  bool reset) {
    (void)n;
    if (reset)
        k_arrive_reset<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.c_arrive,
                                                                   ws.climb_next);
    const int g = climb_grid<100>((const void *)k_collision_climb, ws.leaf_cap);
    k_collision_climb<<<g, kWave, 0, s>>>(
        ws.st, ws.xs, ws.ys, ws.zs, ws.vxs, ws.vys, ws.vzs, ws.rads, dt, ws.ent_cell, ws.c_level,
        ws.c_first, ws.c_count, ws.c_child, ws.c_nchild, ws.c_parent, ws.c_arrive,
        ws.climb_next, ws.ccell,
        ws.c_crmax, ws.ndisks > 1 ? ws.seg : nullptr, ws.disk_L, ws.pcol);
    k_pack_collision<<<cell_grid(ws.cell_cap, 256), 256, 0, s>>>(ws.st, ws.ccell, ws.c_count,
                                                                 ws.c_child, ws.c_nchild, ws.wc,
                                                                 ws.c_entry, ws.c_nent, ws.c_first);
    return hipGetLastError();
}

}  // namespace ncorp

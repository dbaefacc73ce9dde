// Downward pass (Eq. 26) and evaluation at the moonlets: direct sums of the
// walk's brute-force pairs plus the leaf expansion.
//
// Descent: C^(m)(s_1) = sum_{|b| <= p-m} C_{a+b}(s_0) (s_1 - s_0)^b / b!.  Applied
// from the root down the paper's way, every leaf ends up with the sum of its own
// and its ancestors' walk tensors, each shifted to the leaf's centre; that sum is
// formed directly per leaf (shifts compose exactly), so no pass waits on another.
//
// Evaluation: one wave per leaf.  Its sources (every cell the walk paired with
// the leaf or one of its ancestors for a direct sum) are prefix-summed into one
// flat range and streamed through LDS 256 moonlets at a time; leaves with fewer
// than 64 moonlets split each tile over lane groups.  In the FP32-bulk form offsets from the leaf centre are formed in
// FP64 and rounded, each source tile is summed in FP32, and the tile sums are
// added with Kahan compensation.  The leaf's C tensors then give
// a_i += sum_{|b| <= p-1} C_{e+b}(s_leaf) (x_i - s_leaf)^b / b!.
#include "ncorp_internal.h"

namespace ncorp {

template <int P>
__device__ __forceinline__ void scaled_pow(double ux, double uy, double uz, double *px,
                                           double *py, double *pz) {
    px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
    for (int a = 1; a <= P; a++) {
        const double inv = 1.0 / (double)a;
        px[a] = px[a - 1] * ux * inv;
        py[a] = py[a - 1] * uy * inv;
        pz[a] = pz[a - 1] * uz * inv;
    }
}

// Descent without inter-cell waiting.  Shifting a degree-p local expansion is an
// exact re-expansion, so shifts compose: C(leaf) = sum over the leaf and its
// ancestors a of shift(C_walk(a), s_leaf - s_a).  One thread per (leaf, output
// order m) sums that chain; threads are ordered by m so a wave runs one order.
template <int P, int M>
__device__ __forceinline__ void leaf_local_order(int cl, const int32_t *__restrict__ c_parent,
                                                 const double4 *__restrict__ gcell,
                                                 const double *__restrict__ local,
                                                 const int32_t *__restrict__ m2l_cnt,
                                                 double *__restrict__ out) {
    constexpr int NL = n_local(P), NR = P - M, NC = ncomp(M);
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; k++) acc[k] = 0.0;
    const double4 gl = gcell[cl];
    int a = cl;
    for (int up = 0; up <= kMaxDepth && a >= 0; up++) {
        if (m2l_cnt[a] != 0) {                       // cells without M2L hold zeros
            const double4 ga = gcell[a];
            double px[NR + 1], py[NR + 1], pz[NR + 1];
            scaled_pow<NR>(gl.x - ga.x, gl.y - ga.y, gl.z - ga.z, px, py, pz);
            const double *ca = local + (int64_t)a * NL;
#pragma unroll
            for (int b = 0; b <= M; b++)
#pragma unroll
                for (int c = 0; c <= M - b; c++) {
                    const int aa = M - b - c;
                    double sum = acc[tri(b + c) + c];
#pragma unroll
                    for (int n = 0; n <= NR; n++)
#pragma unroll
                        for (int b2 = 0; b2 <= n; b2++)
#pragma unroll
                            for (int c2 = 0; c2 <= n - b2; c2++) {
                                const int a2 = n - b2 - c2;
                                sum += ca[cidx(aa + a2, b + b2, c + c2)] *
                                       (px[a2] * py[b2] * pz[c2]);
                            }
                    acc[tri(b + c) + c] = sum;
                }
        }
        a = c_parent[a];
    }
#pragma unroll
    for (int k = 0; k < NC; k++) out[cidx(M, 0, 0) + k] = acc[k];
}

template <int P>
__global__ void __launch_bounds__(128)
k_leaf_local(const DevState *__restrict__ st, const int32_t *__restrict__ ent_cell,
             const int32_t *__restrict__ c_parent, const double4 *__restrict__ gcell,
             const double *__restrict__ local, const int32_t *__restrict__ m2l_cnt,
             double *__restrict__ cleaf) {
    constexpr int NL = n_local(P);
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    const int64_t total = (int64_t)K * P;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(t / K) + 1, e = (int)(t % K);
        const int cl = ent_cell[e];
        double *out = cleaf + (int64_t)e * NL;
        switch (m) {
            case 1: leaf_local_order<P, 1>(cl, c_parent, gcell, local, m2l_cnt, out); break;
            case 2: if constexpr (P >= 2) leaf_local_order<P, (P >= 2 ? 2 : 1)>(cl, c_parent, gcell, local, m2l_cnt, out); break;
            case 3: if constexpr (P >= 3) leaf_local_order<P, (P >= 3 ? 3 : 1)>(cl, c_parent, gcell, local, m2l_cnt, out); break;
            case 4: if constexpr (P >= 4) leaf_local_order<P, (P >= 4 ? 4 : 1)>(cl, c_parent, gcell, local, m2l_cnt, out); break;
            case 5: if constexpr (P >= 5) leaf_local_order<P, (P >= 5 ? 5 : 1)>(cl, c_parent, gcell, local, m2l_cnt, out); break;
            case 6: if constexpr (P >= 6) leaf_local_order<P, (P >= 6 ? 6 : 1)>(cl, c_parent, gcell, local, m2l_cnt, out); break;
            default: break;
        }
    }
}

// ------------------------------------------------------------------ evaluation
template <typename T> struct Acc3;
template <> struct Acc3<double> {
    double x = 0, y = 0, z = 0;
    __device__ void add_tile(double px, double py, double pz) { x += px; y += py; z += pz; }
    __device__ void fold(double &ox, double &oy, double &oz) const { ox = x; oy = y; oz = z; }
};
// Kahan-compensated FP32 sums of FP32 tile partials
template <> struct Acc3<float> {
    float x = 0, y = 0, z = 0, cx = 0, cy = 0, cz = 0;
    __device__ static void kahan(float &s, float &c, float v) {
        float yv = v - c;
        float t = s + yv;
        c = (t - s) - yv;
        s = t;
    }
    __device__ void add_tile(float px, float py, float pz) {
        kahan(x, cx, px); kahan(y, cy, py); kahan(z, cz, pz);
    }
    __device__ void fold(double &ox, double &oy, double &oz) const {
        ox = (double)x - (double)cx; oy = (double)y - (double)cy; oz = (double)z - (double)cz;
    }
};

__device__ __forceinline__ int wave_excl_sum_p(int v, int lane, int &total) {
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(x, o);
        if (lane >= o) x += t;
    }
    total = __shfl(x, kWave - 1);
    return x - v;
}

template <typename T> __device__ __forceinline__ T rsq(T v);
template <> __device__ __forceinline__ double rsq<double>(double v) { return rsqrt(v); }
template <> __device__ __forceinline__ float rsq<float>(float v) { return rsqrtf(v); }
template <typename T> __device__ __forceinline__ T fmat(T a, T b, T c);
template <> __device__ __forceinline__ double fmat<double>(double a, double b, double c) { return fma(a, b, c); }
template <> __device__ __forceinline__ float fmat<float>(float a, float b, float c) { return fmaf(a, b, c); }

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
// r^2 floor: a moonlet meets itself (dx = 0) in its own leaf; the floor keeps
// 1/r^3 finite there so the term is exactly 0, and is far below any pair distance
// (FP32: added to r^2; FP64: a lower bound on r^2).  m / floor^(3/2) stays finite for
// G m up to ~3e11 (FP32) and ~1e158 (FP64).
template <typename T> __device__ __forceinline__ T r2_floor();
template <> __device__ __forceinline__ float r2_floor<float>() { return 1e-18f; }
template <> __device__ __forceinline__ double r2_floor<double>() { return 1e-100; }

constexpr int kP2PTile = 256;       // source moonlets staged per LDS tile (default)
constexpr int kP2PSrc = kWave;      // source cells per batch, one per lane (prefix sums in LDS)

// Exclusive prefix sums of the moonlet counts of a batch's source cells (one per
// lane) into s_pref[0..kP2PSrc]; returns the total.
__device__ __forceinline__ int batch_prefix(int cnt, int32_t *s_pref, int lane) {
    int tot;
    const int ex = wave_excl_sum_p(cnt, lane, tot);
    s_pref[lane] = ex;
    if (lane == 0) s_pref[kP2PSrc] = tot;
    return tot;
}

// One source against the NT targets a lane holds.
template <typename T, int NT>
__device__ __forceinline__ void interact(const typename Vec4<T>::type &v, const T (&xi)[NT],
                                         const T (&yi)[NT], const T (&zi)[NT], T (&px)[NT],
                                         T (&py)[NT], T (&pz)[NT]) {
    const T floor2 = r2_floor<T>();
#pragma unroll
    for (int k = 0; k < NT; k++) {
        const T dx = v.x - xi[k], dy = v.y - yi[k], dz = v.z - zi[k];
        T rinv;
        if constexpr (sizeof(T) == 4) {
            // the floor enters as an addend, so r2 >= 1e-24 is a normal float and the
            // hardware reciprocal square root needs no denormal handling
            const T r2 = fmat<T>(dz, dz, fmat<T>(dy, dy, fmat<T>(dx, dx, floor2)));
            rinv = __builtin_amdgcn_rsqf(r2);
        } else {
            T r2 = fmat<T>(dz, dz, fmat<T>(dy, dy, dx * dx));
            r2 = r2 > floor2 ? r2 : floor2;
            rinv = rsq<T>(r2);
        }
        const T w = v.w * (rinv * rinv) * rinv;
        px[k] = fmat<T>(dx, w, px[k]);
        py[k] = fmat<T>(dy, w, py[k]);
        pz[k] = fmat<T>(dz, w, pz[k]);
    }
}

// Direct sums of the NT targets a lane holds over a batch of source cells whose
// moonlet ranges are s_first[k] .. + (s_pref[k+1] - s_pref[k]), k < nsb, tot
// moonlets in all; the batch is streamed through LDS TILE moonlets at a time and
// the lane's group takes sources j0, j0 + G, ... of every tile.
template <typename T, int NT, int TILE>
__device__ __forceinline__ void p2p_batch(int tot, int nsb, const int32_t *s_first,
                                          const int32_t *s_pref,
                                          typename Vec4<T>::type *tile,
                                          const double *__restrict__ xs,
                                          const double *__restrict__ ys,
                                          const double *__restrict__ zs,
                                          const double *__restrict__ mus, const double4 g,
                                          const T (&xi)[NT], const T (&yi)[NT], const T (&zi)[NT],
                                          int j0, int G, Acc3<T> (&acc)[NT]) {
    using V = typename Vec4<T>::type;
    const int lane = threadIdx.x & (kWave - 1);
    for (int p0 = 0; p0 < tot; p0 += TILE) {
        const int nj = tot - p0 < TILE ? tot - p0 : TILE;
        // stage the tile: source moonlet q of the batch -> its cell by binary
        // search over the prefix sums
#pragma unroll
        for (int k = 0; k < TILE / 64; k++) {
            const int q = p0 + lane + 64 * k;
            if (q < tot) {
                int lo = 0, hi = nsb;          // s_pref[lo] <= q < s_pref[hi]
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pref[mid] <= q) lo = mid; else hi = mid;
                }
                const int j = s_first[lo] + (q - s_pref[lo]);
                V v;
                v.x = (T)(xs[j] - g.x);
                v.y = (T)(ys[j] - g.y);
                v.z = (T)(zs[j] - g.z);
                v.w = (T)mus[j];
                tile[lane + 64 * k] = v;
            }
        }
        wave_sync();
        T px[NT], py[NT], pz[NT];
#pragma unroll
        for (int k = 0; k < NT; k++) px[k] = py[k] = pz[k] = (T)0;
        if constexpr (NT == 1) {
#pragma unroll 4
            for (int j = j0; j < nj; j += G) interact<T, NT>(tile[j], xi, yi, zi, px, py, pz);
        } else if constexpr (NT == 2) {
#pragma unroll 2
            for (int j = j0; j < nj; j += G) interact<T, NT>(tile[j], xi, yi, zi, px, py, pz);
        } else {
            for (int j = j0; j < nj; j += G) interact<T, NT>(tile[j], xi, yi, zi, px, py, pz);
        }
#pragma unroll
        for (int k = 0; k < NT; k++) acc[k].add_tile(px[k], py[k], pz[k]);
        wave_sync();
    }
}

// Direct sums for ntc <= 64 targets (moonlets tb .. tb+ntc-1) of one leaf, over
// the whole list (one LDS batch) or over its batches b0, b0 + bstep, ... of
// kP2PSrc source cells.  The lanes form G = 64 / lpg groups of lpg = ceil(ntc / NT)
// lanes; lane li of a group holds targets li and li + lpg (NT = 2), and the groups
// split every tile's sources.  The group partials are added in group order and
// written to out[d * n + i], d = x, y, z.
template <typename T, int NT, int TILE>
__device__ __forceinline__ void p2p_targets(int ntc, int tb, bool one, int tot1, int len,
                                            int b0, int bstep,
                                            const int32_t *__restrict__ list, int32_t *s_first,
                                            int32_t *s_pref, typename Vec4<T>::type *tile,
                                            const double *__restrict__ xs,
                                            const double *__restrict__ ys,
                                            const double *__restrict__ zs,
                                            const double *__restrict__ mus,
                                            const int32_t *__restrict__ c_first,
                                            const int32_t *__restrict__ c_count, const double4 g,
                                            double *__restrict__ out, int64_t n) {
    const int lane = threadIdx.x & (kWave - 1);
    const int lpg = (ntc + NT - 1) / NT;
    const int G = kWave / lpg;
    const int grp = lane / lpg, li = lane % lpg;
    T xi[NT], yi[NT], zi[NT];
#pragma unroll
    for (int k = 0; k < NT; k++) {
        const int t = li + k * lpg;
        const int i = tb + (t < ntc ? t : 0);
        xi[k] = (T)(xs[i] - g.x);
        yi[k] = (T)(ys[i] - g.y);
        zi[k] = (T)(zs[i] - g.z);
    }
    const int j0 = grp < G ? grp : TILE;           // lanes beyond the groups idle
    Acc3<T> acc[NT];
    if (one) {
        p2p_batch<T, NT, TILE>(tot1, len, s_first, s_pref, tile, xs, ys, zs, mus, g, xi, yi, zi, j0,
                         G, acc);
    } else {
        for (int sb = b0 * kP2PSrc; sb < len; sb += bstep * kP2PSrc) {
            const int nsb = len - sb < kP2PSrc ? len - sb : kP2PSrc;
            wave_sync();
            int cf = 0, cn = 0;
            if (lane < nsb) {
                const int B = list[sb + lane];
                cf = c_first[B];
                cn = c_count[B];
            }
            s_first[lane] = cf;
            const int tot = batch_prefix(cn, s_pref, lane);
            wave_sync();
            p2p_batch<T, NT, TILE>(tot, nsb, s_first, s_pref, tile, xs, ys, zs, mus, g, xi, yi, zi,
                             j0, G, acc);
        }
    }
    // add the partials of groups 1 .. G-1 to group 0's, in group order
#pragma unroll
    for (int k = 0; k < NT; k++) {
        double px, py, pz;                     // this lane's partials
        acc[k].fold(px, py, pz);
        double ox = px, oy = py, oz = pz;
        for (int gi = 1; gi < G; gi++) {
            const int src = gi * lpg + li;
            ox += __shfl(px, src);
            oy += __shfl(py, src);
            oz += __shfl(pz, src);
        }
        const int t = li + k * lpg;
        if (grp == 0 && t < ntc) {
            out[tb + t] = ox;
            out[n + tb + t] = oy;
            out[2 * n + tb + t] = oz;
        }
    }
}

// Targets per lane for a chunk of ntc <= 64 targets: lpg = ceil(ntc / NT) lanes hold
// them, G = 64 / lpg lane groups split every tile, so a round keeps ntc * G of the
// 64 * NT lane slots busy.  The NT in 1..4 with the largest share wins (the smaller
// on ties): 43 targets use 3 per lane (4 groups of 15 lanes, 90 % busy) where one or
// two per lane leave a third of the lanes idle.
__device__ __forceinline__ int targets_per_lane(int ntc, int tmax) {
    int best = 1, best_score = -1;
#pragma unroll
    for (int nt = 1; nt <= 4; nt++) {
        if (nt > tmax) break;
        const int lpg = (ntc + nt - 1) / nt;
        const int score = ntc * (kWave / lpg) * (12 / nt);
        if (score > best_score) { best = nt; best_score = score; }
    }
    return best;
}

template <typename T, int TILE>
__device__ __forceinline__ void p2p_targets_any(int ntc, int tmax, int tb, bool one, int tot1,
                                                int len, int b0, int bstep,
                                                const int32_t *__restrict__ list,
                                                int32_t *s_first, int32_t *s_pref,
                                                typename Vec4<T>::type *tile,
                                                const double *__restrict__ xs,
                                                const double *__restrict__ ys,
                                                const double *__restrict__ zs,
                                                const double *__restrict__ mus,
                                                const int32_t *__restrict__ c_first,
                                                const int32_t *__restrict__ c_count,
                                                const double4 g, double *__restrict__ out,
                                                int64_t n) {
    switch (targets_per_lane(ntc, tmax)) {
        case 1:
            p2p_targets<T, 1, TILE>(ntc, tb, one, tot1, len, b0, bstep, list, s_first, s_pref, tile,
                              xs, ys, zs, mus, c_first, c_count, g, out, n);
            break;
        case 2:
            p2p_targets<T, 2, TILE>(ntc, tb, one, tot1, len, b0, bstep, list, s_first, s_pref, tile,
                              xs, ys, zs, mus, c_first, c_count, g, out, n);
            break;
        case 3:
            p2p_targets<T, 3, TILE>(ntc, tb, one, tot1, len, b0, bstep, list, s_first, s_pref, tile,
                              xs, ys, zs, mus, c_first, c_count, g, out, n);
            break;
        default:
            p2p_targets<T, 4, TILE>(ntc, tb, one, tot1, len, b0, bstep, list, s_first, s_pref, tile,
                              xs, ys, zs, mus, c_first, c_count, g, out, n);
            break;
    }
}

constexpr int kP2PWaves = 4;        // independent waves per block
static_assert(kP2PListLDS == kP2PSrc, "one LDS batch holds a list the pre-pass leaves unsorted");

// Direct sums of every leaf, one wave per work item.  A leaf whose source list fits
// one LDS batch is one item.  A leaf whose list is longer (the pre-pass sorted it)
// would keep a single wave busy long after all others finished, so it is split over
// kLongSlots items: item `slot` takes the batches slot, slot + kLongSlots, ... and
// writes its partial sums to part[slot], which the evaluation kernel adds in slot
// order.  The split items come first, so they start first and the short leaves fill
// in around them within the same launch.
template <typename T, int TILE>
__global__ void __launch_bounds__(kWave * kP2PWaves)
k_p2p(const DevState *__restrict__ st, const double *__restrict__ xs,
      const double *__restrict__ ys, const double *__restrict__ zs,
      const double *__restrict__ mus, const int32_t *__restrict__ ent_cell,
      const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
      const double4 *__restrict__ gcell, const int32_t *__restrict__ p2p_cnt,
      int32_t *__restrict__ p2p_seg, int stride, const int32_t *__restrict__ longs,
      double *__restrict__ part, double *__restrict__ acc_s, int64_t n, int tmax) {
    using V = typename Vec4<T>::type;
    static_assert(TILE >= 128 && TILE % 64 == 0, "the tile doubles as the sort's scratch");
    __shared__ __align__(16) V tiles[kP2PWaves][TILE];
    __shared__ int32_t firsts[kP2PWaves][kP2PSrc], prefs[kP2PWaves][kP2PSrc + 1];
    if (st->status & kSkipMask) return;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    V *tile = tiles[wid];
    int32_t *s_first = firsts[wid], *s_pref = prefs[wid];
    // the tile doubles as sort scratch before any moonlet is staged
    int32_t *scratch = reinterpret_cast<int32_t *>(tile);
    const int K = st->nleaves;
    const int nlong = st->nlong_p2p * kLongSlots;
    for (int w = blockIdx.x * kP2PWaves + wid; w < nlong + K; w += gridDim.x * kP2PWaves) {
        if (w < nlong) {
            const int e = longs[w / kLongSlots], slot = w % kLongSlots;
            const int c = ent_cell[e];
            const int f = c_first[c], nt = c_count[c];
            const double4 g = gcell[c];
            const int32_t *list = p2p_seg + (int64_t)e * stride;
            const int len = p2p_cnt[e];
            double *out = part + (int64_t)slot * 3 * n;
            wave_sync();                              // this wave's LDS is free again
            for (int t0 = 0; t0 < nt; t0 += kWave) {
                const int ntc = nt - t0 < kWave ? nt - t0 : kWave;
                p2p_targets_any<T, TILE>(ntc, tmax, f + t0, false, 0, len, slot, kLongSlots,
                                         list, s_first, s_pref, tile, xs, ys, zs, mus, c_first,
                                         c_count, g, out, n);
            }
            continue;
        }
        const int e = w - nlong;
        const int c = ent_cell[e];
        const int f = c_first[c], nt = c_count[c];
        const double4 g = gcell[c];
        int32_t *list = p2p_seg + (int64_t)e * stride;
        const int len = p2p_cnt[e];
        if (len > kP2PSrc) continue;                  // split into the items above
        wave_sync();                                  // this wave's LDS is free again
        // one batch: rank the sources in LDS and place each source's moonlet range
        // at its rank directly
        const int v = lane < len ? list[lane] : 0x7fffffff;
        const int cf = lane < len ? c_first[v] : 0;
        const int cn = lane < len ? c_count[v] : 0;
        scratch[lane] = v;
        wave_sync();
        if (lane < len) {
            const int4 *s4 = reinterpret_cast<const int4 *>(scratch);
            int rk = 0;
#pragma unroll
            for (int j = 0; j < kP2PSrc / 4; j++) {
                const int4 t = s4[j];
                rk += (t.x < v) + (t.y < v) + (t.z < v) + (t.w < v);
            }
            s_first[rk] = cf;
            s_pref[rk] = cn;
        }
        wave_sync();
        const int c1 = lane < len ? s_pref[lane] : 0;
        wave_sync();
        const int tot1 = batch_prefix(c1, s_pref, lane);
        wave_sync();
        for (int t0 = 0; t0 < nt; t0 += kWave) {
            const int ntc = nt - t0 < kWave ? nt - t0 : kWave;
            p2p_targets_any<T, TILE>(ntc, tmax, f + t0, true, tot1, len, 0, 1, list, s_first,
                                     s_pref, tile, xs, ys, zs, mus, c_first, c_count, g, acc_s,
                                     n);
        }
    }
}

// evaluation of the leaf's expansion at its moonlets (Eq. 26 down to C^(1)),
// added to the direct sums and written in input order
constexpr int kL2PWaves = 4;        // independent waves per block

template <int P>
__global__ void __launch_bounds__(kWave * kL2PWaves)
k_l2p(const DevState *__restrict__ st, const double *__restrict__ xs,
      const double *__restrict__ ys, const double *__restrict__ zs,
      const uint32_t *__restrict__ perm, const int32_t *__restrict__ ent_cell,
      const int32_t *__restrict__ c_first, const int32_t *__restrict__ c_count,
      const double4 *__restrict__ gcell, const double *__restrict__ cleaf,
      const double *__restrict__ acc_s, const int32_t *__restrict__ p2p_cnt,
      const double *__restrict__ part, int64_t n, double *__restrict__ ax,
      double *__restrict__ ay, double *__restrict__ az, double4 *__restrict__ acc4) {
    constexpr int NL = n_local(P);
    if (st->status & kSkipMask) return;
    const int K = st->nleaves;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    for (int e = blockIdx.x * kL2PWaves + wid; e < K; e += gridDim.x * kL2PWaves) {
        const int c = ent_cell[e];
        const int f = c_first[c], nt = c_count[c];
        const double4 g = gcell[c];
        const bool longlist = p2p_cnt[e] > kP2PListLDS;   // direct sums in kLongSlots parts
        // the leaf's C is wave-uniform: scalar loads, no copy in LDS
        const double *__restrict__ cle = cleaf + (int64_t)__builtin_amdgcn_readfirstlane(e) * NL;
        for (int t0 = 0; t0 < nt; t0 += 64) {
            const int t = t0 + lane;
            if (t >= nt) continue;
            const int i = f + t;
            double px[P], py[P], pz[P];
            const double ux = xs[i] - g.x, uy = ys[i] - g.y, uz = zs[i] - g.z;
            px[0] = py[0] = pz[0] = 1.0;
#pragma unroll
            for (int a = 1; a < P; a++) {
                const double inv = 1.0 / (double)a;
                px[a] = px[a - 1] * ux * inv;
                py[a] = py[a - 1] * uy * inv;
                pz[a] = pz[a - 1] * uz * inv;
            }
            double lx = 0.0, ly = 0.0, lz = 0.0;
#pragma unroll
            for (int nn = 0; nn < P; nn++)
#pragma unroll
                for (int b2 = 0; b2 <= nn; b2++)
#pragma unroll
                    for (int c2 = 0; c2 <= nn - b2; c2++) {
                        const int a2 = nn - b2 - c2;
                        const double w = px[a2] * py[b2] * pz[c2];
                        lx += cle[cidx(1 + a2, b2, c2)] * w;
                        ly += cle[cidx(a2, 1 + b2, c2)] * w;
                        lz += cle[cidx(a2, b2, 1 + c2)] * w;
                    }
            double dx = 0.0, dy = 0.0, dz = 0.0;       // direct sums
            if (longlist) {
#pragma unroll
                for (int sl = 0; sl < kLongSlots; sl++) {
                    const double *ps = part + (int64_t)sl * 3 * n;
                    dx += ps[i];
                    dy += ps[n + i];
                    dz += ps[2 * n + i];
                }
            } else {
                dx = acc_s[i];
                dy = acc_s[n + i];
                dz = acc_s[2 * n + i];
            }
            const uint32_t o = perm[i];
            if (acc4) {
                acc4[o] = make_double4(dx + lx, dy + ly, dz + lz, 0.0);
            } else {
                ax[o] = dx + lx;
                ay[o] = dy + ly;
                az[o] = dz + lz;
            }
        }
    }
}

template <int P>
static void launch_leaf_local(const Workspace &ws, hipStream_t s) {
    int64_t g = ((int64_t)ws.n_max * P + 127) / 128;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    k_leaf_local<P><<<(int)g, 128, 0, s>>>(ws.st, ws.ent_cell, ws.c_parent, ws.gcell, ws.local,
                                           ws.m2l_cnt, ws.cleaf);
}

hipError_t launch_l2l(const Workspace &ws, int p, hipStream_t s) {
    switch (p) {
        case 1: launch_leaf_local<1>(ws, s); break;
        case 2: launch_leaf_local<2>(ws, s); break;
        case 3: launch_leaf_local<3>(ws, s); break;
        case 4: launch_leaf_local<4>(ws, s); break;
        case 5: launch_leaf_local<5>(ws, s); break;
        case 6: launch_leaf_local<6>(ws, s); break;
        default: break;
    }
    return hipGetLastError();
}

template <typename T, int TILE>
static void launch_p2p_t(const Workspace &ws, int64_t n, int tmax, hipStream_t s) {
    // one item per leaf plus kLongSlots - 1 more per long leaf; the grid strides
    int64_t g = (ws.leaf_cap + kP2PWaves - 1) / kP2PWaves + kLongGrid;
    g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
    k_p2p<T, TILE><<<(int)g, kWave * kP2PWaves, 0, s>>>(
        ws.st, ws.xs, ws.ys, ws.zs, ws.mus, ws.ent_cell, ws.c_first, ws.c_count, ws.gcell,
        ws.p2p_cnt, ws.p2p_seg, ws.p2p_stride, ws.long_p2p, ws.p2p_part, ws.acc_s, n, tmax);
}

template <typename T>
static void launch_p2p_tile(const Workspace &ws, int64_t n, int tile, int tmax, hipStream_t s) {
    switch (tile) {
        case 128: launch_p2p_t<T, 128>(ws, n, tmax, s); break;
        case 512: launch_p2p_t<T, 512>(ws, n, tmax, s); break;
        default: launch_p2p_t<T, kP2PTile>(ws, n, tmax, s); break;
    }
}

// tile: source moonlets per LDS tile (128, 256, 512; 0 = 256); tmax: most targets per
// lane (1..4; 0 = 4)
hipError_t launch_p2p(const Workspace &ws, int64_t n, int precision, int tile, int tmax,
                      hipStream_t s) {
    const int tm = tmax > 0 ? tmax : 4;
    if (precision == NCORP_FP32_BULK) launch_p2p_tile<float>(ws, n, tile, tm, s);
    else launch_p2p_tile<double>(ws, n, tile, tm, s);
    return hipGetLastError();
}

template <int P>
static void launch_l2p_p(const Workspace &ws, int64_t n, double *ax, double *ay, double *az,
                         hipStream_t s, double4 *acc4) {
    int64_t g = (ws.leaf_cap + kL2PWaves - 1) / kL2PWaves;
    g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
    k_l2p<P><<<(int)g, kWave * kL2PWaves, 0, s>>>(ws.st, ws.xs, ws.ys, ws.zs, ws.idx, ws.ent_cell, ws.c_first,
                              ws.c_count, ws.gcell, ws.cleaf, ws.acc_s, ws.p2p_cnt, ws.p2p_part, n,
                              ax, ay, az, acc4);
}

hipError_t launch_l2p(const Workspace &ws, int64_t n, int p, double *ax, double *ay, double *az,
                      hipStream_t s, double4 *acc4) {
    switch (p) {
        case 1: launch_l2p_p<1>(ws, n, ax, ay, az, s, acc4); break;
        case 2: launch_l2p_p<2>(ws, n, ax, ay, az, s, acc4); break;
        case 3: launch_l2p_p<3>(ws, n, ax, ay, az, s, acc4); break;
        case 4: launch_l2p_p<4>(ws, n, ax, ay, az, s, acc4); break;
        case 5: launch_l2p_p<5>(ws, n, ax, ay, az, s, acc4); break;
        case 6: launch_l2p_p<6>(ws, n, ax, ay, az, s, acc4); break;
        default: break;
    }
    return hipGetLastError();
}

}  // namespace ncorp

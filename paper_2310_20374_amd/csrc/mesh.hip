// Mesh module (Sect. 3.3): mutual gravity and collision search restricted to
// moonlets in each other's neighbourhood on a mesh of cubic cells of side gamma,
// plus the moonlets that interact with everyone (too large for the mesh, and for
// gravity the three most massive).
//
// Build: every moonlet gets its cell c = floor(r / gamma); the moonlets are sorted
// by the Morton key of their cell with a stable radix sort (input order inside a
// cell; moonlets kept out of the mesh get the largest key and end up last), so each
// occupied cell is one run of the sorted array and nearby cells sit close together.
// Each run is recorded as the cell's range [start, end): in a dense grid over the
// box of occupied cells when that box fits the grid buffer (32 cells per moonlet of
// capacity), else in an open-addressing hash table keyed by the cell's Morton key
// (linear probing, at most half full).  A neighbourhood scan looks up the 27 cells around a moonlet's cell and
// reads their moonlets: exactly the neighbours, no other cell shares an entry.  The
// lanes of a wave hold neighbouring moonlets and look up overlapping cells.
//
// The mesh size: Eq. (4) at the first mesh (or the value given), then Eq. (6) from
// the neighbour count of the previous mesh, kept on the device so that a step
// loop (and a captured graph of it) needs no host round trip.
#include <climits>

#include "contact.h"

namespace ncorp {
namespace {

constexpr int kMeshBlock = 256;
constexpr int kMeshTopBlocks = 256;
constexpr int kMeshChunks = 64;      // source chunks of the all-pairs sums
constexpr int kMeshBigRows = 16;     // big moonlets handled side by side

// 21 bits of v spread to every third bit
__device__ __forceinline__ unsigned long long spread3(unsigned long long v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// every third bit of v (from bit 0) packed into 21 bits: the inverse of spread3
__device__ __forceinline__ unsigned long long compact3(unsigned long long v) {
    v &= 0x1249249249249249ull;
    v = (v | (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v | (v >> 4)) & 0x100f00f00f00f00full;
    v = (v | (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v | (v >> 16)) & 0x1f00000000ffffull;
    v = (v | (v >> 32)) & 0x1fffffull;
    return v;
}

// Morton key of a cell (coordinates within +-kMeshCellLimit)
__device__ __forceinline__ unsigned long long cell_key(int x, int y, int z) {
    return spread3((unsigned)(x + kMeshCellLimit)) |
           (spread3((unsigned)(y + kMeshCellLimit)) << 1) |
           (spread3((unsigned)(z + kMeshCellLimit)) << 2);
}

// table slot where the probe for a key starts (a 64-bit mixing step, then the
// table's power-of-two mask)
__device__ __forceinline__ int64_t slot_of(unsigned long long k, int64_t mask) {
    k ^= k >> 31;
    k *= 0x7fb5d329728ea185ull;
    k ^= k >> 27;
    k *= 0x81dadef4bc2dd44dull;
    k ^= k >> 33;
    return (int64_t)(k & (unsigned long long)mask);
}

// range of the moonlets of a cell, (0, 0) if it holds none
__device__ __forceinline__ int2 lookup(const MeshSlot *__restrict__ tab, int64_t mask,
                                      unsigned long long k) {
    int64_t h = slot_of(k, mask);
    for (int64_t probes = 0; probes <= mask; probes++) {
        const MeshSlot e = tab[h];
        if (e.key == k) return make_int2(e.start, e.end);
        if (e.key == kMeshEmpty) break;
        h = (h + 1) & mask;
    }
    return make_int2(0, 0);
}

// cell of a position; false if a coordinate reaches +-(kMeshCellLimit - 1)
__device__ __forceinline__ bool cell_of(double x, double y, double z, double g, int4 &c) {
    const double fx = floor(x / g), fy = floor(y / g), fz = floor(z / g);
    const double lim = (double)(kMeshCellLimit - 1);  // neighbours stay in 21 bits
    if (!(fabs(fx) < lim && fabs(fy) < lim && fabs(fz) < lim)) return false;
    c.x = (int)fx; c.y = (int)fy; c.z = (int)fz; c.w = 0;
    return true;
}

__device__ __forceinline__ void add_pull(double4 src, double x, double y, double z, double &a0,
                                         double &a1, double &a2) {
    const double dx = src.x - x, dy = src.y - y, dz = src.z - z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 == 0.0) return;
    const double r = sqrt(r2);
    const double f = src.w / (r2 * r);          // one division per pair
    a0 += f * dx;
    a1 += f * dy;
    a2 += f * dz;
}

// How a scan finds the moonlets of a cell: directly in the dense grid of the box of
// occupied cells when that box fits the grid buffer (neighbouring cells then sit next
// to each other in memory), else through the hash table.  Cells outside the box are
// empty.
struct CellIndex {
    const int2 *grid;
    const MeshSlot *tab;
    int64_t mask;
    int x0, y0, z0, dx, dy, dz;
    bool dense;
};

__device__ __forceinline__ CellIndex cell_index(const MeshState *__restrict__ ms,
                                                const int2 *grid, const MeshSlot *tab,
                                                int64_t mask) {
    CellIndex ci;
    ci.grid = grid; ci.tab = tab; ci.mask = mask;
    ci.x0 = ms->box_x0; ci.y0 = ms->box_y0; ci.z0 = ms->box_z0;
    ci.dx = ms->box_dx; ci.dy = ms->box_dy; ci.dz = ms->box_dz;
    ci.dense = ms->dense != 0;
    return ci;
}

__device__ __forceinline__ int2 cell_range(const CellIndex &ci, int x, int y, int z) {
    if (ci.dense) {
        const int ix = x - ci.x0, iy = y - ci.y0, iz = z - ci.z0;
        if ((unsigned)ix >= (unsigned)ci.dx || (unsigned)iy >= (unsigned)ci.dy ||
            (unsigned)iz >= (unsigned)ci.dz)
            return make_int2(0, 0);
        return ci.grid[ix + (int64_t)ci.dx * (iy + (int64_t)ci.dy * iz)];
    }
    return lookup(ci.tab, ci.mask, cell_key(x, y, z));
}

// sum of v over the block, valid in thread 0 (every thread calls it)
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / kWave); k++) t += red[k];
    __syncthreads();
    return t;
}

// the neighbour count of the current mesh, from the scan's per-block partials
__global__ void __launch_bounds__(1024)
k_mesh_count_done(const unsigned long long *__restrict__ part, int64_t n, MeshState *ms) {
    __shared__ unsigned long long red[1024 / kWave];
    unsigned long long v = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) v += part[i];
    const unsigned long long t = block_sum_u64(v, red);
    if (threadIdx.x == 0) {
        ms->nbr_sum = t;
        ms->measured = 1;
    }
}

// ------------------------------------------------------------------ build
__global__ void k_mesh_clear_state(MeshState *ms) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MeshState z = {};
        *ms = z;
    }
}

// Start of a build: when the last build was dense and completed, its cells are the
// only non-zero entries of the grid buffer and their indices are still its sorted
// keys, so clearing those entries leaves the whole buffer zero (O(N) instead of the
// box).  grid_sparse is only read here; k_mesh_box resets it after this launch.
__global__ void k_mesh_unset(MeshState *ms, const uint64_t *__restrict__ keys, int2 *grid,
                             int64_t grid_n) {
    const bool sparse = ms->grid_sparse != 0;
    const int64_t m = sparse ? ms->prev_n : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) ms->grid_zero = sparse ? 1 : 0;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < m;
         q += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[q];
        if (k < (uint64_t)grid_n && (q == 0 || keys[q - 1] != k)) grid[k] = make_int2(0, 0);
    }
}

// Clears the cell index of the new mesh.  With the dense grid, also replaces each
// Morton key by the cell's grid index (empty: dense_empty, above every index), so
// that the sort needs only the digits of the grid's size.
__global__ void k_mesh_clear_table(const MeshState *__restrict__ ms, MeshSlot *tab,
                                   int64_t nslots, int2 *grid, int64_t grid_n, uint64_t *keys,
                                   int64_t n, uint64_t dense_empty) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (ms->dense) {
        // unless k_mesh_unset left it zero, the whole buffer (later boxes may be larger
        // than this one, and the next build clears only this build's cells)
        const int64_t nc = ms->grid_zero ? 0 : grid_n;
        for (int64_t b = t0; b < nc; b += stride) grid[b] = make_int2(0, 0);
        const int x0 = ms->box_x0, y0 = ms->box_y0, z0 = ms->box_z0;
        const int64_t dx = ms->box_dx, dy = ms->box_dy;
        for (int64_t i = t0; i < n; i += stride) {
            const unsigned long long k = keys[i];
            if (k == kMeshEmpty) {
                keys[i] = dense_empty;
                continue;
            }
            const int cx = (int)compact3(k) - kMeshCellLimit;
            const int cy = (int)compact3(k >> 1) - kMeshCellLimit;
            const int cz = (int)compact3(k >> 2) - kMeshCellLimit;
            keys[i] = (uint64_t)((cx - x0) + dx * ((cy - y0) + dy * (int64_t)(cz - z0)));
        }
        return;
    }
    for (int64_t b = t0; b < nslots; b += stride) tab[b].key = kMeshEmpty;
}

__global__ void k_mesh_rmax(const double *__restrict__ x, const double *__restrict__ y,
                            const double *__restrict__ z, int64_t n, MeshState *ms) {
    double m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double r2 = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
        m = r2 > m ? r2 : m;       // NaN positions are reported by the keys kernel
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(m, o);
        m = t > m ? t : m;
    }
    // non-negative doubles order like their bit patterns
    if ((threadIdx.x & (kWave - 1)) == 0)
        atomicMax((unsigned long long *)&ms->rmax2, (unsigned long long)__double_as_longlong(m));
}

// the mesh size of the new mesh (Eq. 4 at the first mesh, Eq. 6 after)
__global__ void k_mesh_begin(MeshState *ms, DevState *st, int64_t n, double x_target,
                             double aspect, double rmax, double gamma0, double gamma_min) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double g;
    if (!ms->init) {
        if (gamma0 > 0.0) {
            g = gamma0;
        } else {
            const double R = rmax > 0.0 ? rmax : sqrt(ms->rmax2);
            const double s = aspect * aspect / (1.0 + aspect * aspect);
            g = pow(4.0 * 3.14159265358979323846 * x_target / (81.0 * (double)n), 1.0 / 3.0) *
                pow(s, 1.0 / 6.0) * R;
        }
        ms->init = 1;
    } else if (ms->measured) {
        const double xm = ms->n_in > 0 ? (double)ms->nbr_sum / (double)ms->n_in : 0.0;
        g = xm > 0.0 ? ms->gamma * cbrt(x_target / xm) : 2.0 * ms->gamma;
    } else {
        g = ms->gamma;
    }
    if (g < gamma_min) g = gamma_min;
    if (!(g > 0.0) || !(g < INFINITY)) atomicOr(&st->status, (int32_t)ST_MESH_RANGE);
    ms->gamma = g;
    ms->stamp += 1;
    ms->measured = 0;
    ms->nbr_sum = 0;
    ms->n_in = (int32_t)n;
    ms->ntop = 0;
    ms->nbig = 0;
}

__device__ __forceinline__ int wave_min_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

// minimum over the block (every thread calls it; all get the result)
__device__ __forceinline__ int block_min_i(int v, int *red) {
    v = wave_min_i(v);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    int t = INT_MAX;
    for (int k = 0; k < (int)(blockDim.x / kWave); k++) t = min(t, red[k]);
    __syncthreads();
    return t;
}

// keys (the cell's Morton key; moonlets out of the mesh sorted last) and, per
// block, the box of the cells seen: part[6 b .. 6 b + 5] = min x, y, z, -max x, y, z
__global__ void __launch_bounds__(256)
k_mesh_keys(DevState *st, const MeshState *__restrict__ ms, const double *__restrict__ x,
            const double *__restrict__ y, const double *__restrict__ z,
            const double *__restrict__ R, int64_t n, uint64_t *keys, uint32_t *vals,
            int32_t *box_part, double4 *__restrict__ pack4) {
    __shared__ int red[256 / kWave];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const double g = ms->gamma;
    int4 c = make_int4(INT_MAX, INT_MAX, INT_MAX, 0);
    bool in = false;
    if (i < n) {
        const double px = x[i], py = y[i], pz = z[i];
        pack4[i] = make_double4(px, py, pz, 0.0);   // one record per moonlet for the gather
        uint64_t key = kMeshEmpty;                 // out of the mesh: sorted last
        if (!(2.0 * R[i] > g)) {
            if (cell_of(px, py, pz, g, c)) {
                key = cell_key(c.x, c.y, c.z);
                in = true;
            } else if (isfinite(px) && isfinite(py) && isfinite(pz)) {
                atomicOr(&st->status, (int32_t)ST_MESH_RANGE);
            } else {
                atomicOr(&st->status, (int32_t)ST_NONFINITE);   // kept out: never indexed
            }
        }
        keys[i] = key;
        vals[i] = (uint32_t)i;
    }
    const int mnx = block_min_i(in ? c.x : INT_MAX, red);
    const int mny = block_min_i(in ? c.y : INT_MAX, red);
    const int mnz = block_min_i(in ? c.z : INT_MAX, red);
    const int mxx = block_min_i(in ? -c.x : INT_MAX, red);
    const int mxy = block_min_i(in ? -c.y : INT_MAX, red);
    const int mxz = block_min_i(in ? -c.z : INT_MAX, red);
    if (threadIdx.x == 0) {
        int32_t *b = box_part + 6 * (int64_t)blockIdx.x;
        b[0] = mnx; b[1] = mny; b[2] = mnz; b[3] = mxx; b[4] = mxy; b[5] = mxz;
    }
}

// the box of occupied cells and whether the dense grid holds it
__global__ void __launch_bounds__(1024)
k_mesh_box(const int32_t *__restrict__ box_part, int nblk, MeshState *ms, int64_t grid_cap) {
    __shared__ int red[1024 / kWave];
    int v[6];
    for (int k = 0; k < 6; k++) v[k] = INT_MAX;
    for (int b = threadIdx.x; b < nblk; b += 1024)
        for (int k = 0; k < 6; k++) v[k] = min(v[k], box_part[6 * (int64_t)b + k]);
    for (int k = 0; k < 6; k++) v[k] = block_min_i(v[k], red);
    if (threadIdx.x == 0) {
        ms->grid_sparse = 0;                      // set again by a completed dense build
        if (v[0] == INT_MAX) {                    // no moonlet in the mesh
            ms->box_x0 = ms->box_y0 = ms->box_z0 = 0;
            ms->box_dx = ms->box_dy = ms->box_dz = 0;
            ms->dense = 1;
            return;
        }
        const int64_t dx = (int64_t)(-v[3]) - v[0] + 1, dy = (int64_t)(-v[4]) - v[1] + 1,
                      dz = (int64_t)(-v[5]) - v[2] + 1;
        ms->box_x0 = v[0]; ms->box_y0 = v[1]; ms->box_z0 = v[2];
        const bool dense = dx * dy * dz <= grid_cap;
        ms->box_dx = dense ? (int)dx : 0;
        ms->box_dy = dense ? (int)dy : 0;
        ms->box_dz = dense ? (int)dz : 0;
        ms->dense = dense ? 1 : 0;
    }
}

// sorted positions and cells; the first out-of-mesh position is n_in; the first
// moonlet of every cell claims the cell's slot.  Keys are grid indices (empty:
// dense_empty) with the dense grid, Morton keys (empty: kMeshEmpty) otherwise.
__global__ void k_mesh_runs(DevState *st, MeshState *ms, const uint64_t *__restrict__ keys,
                            const uint32_t *__restrict__ idx, const double4 *__restrict__ pack4,
                            int64_t n, MeshSlot *tab, int64_t mask, int2 *grid, double4 *mpos,
                            int4 *mcell, uint64_t dense_empty) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n || (st->status & kSkipMask)) return;
    const uint32_t i = idx[q];
    const double g = ms->gamma;
    const bool dense = ms->dense != 0;
    const uint64_t empty = dense ? dense_empty : kMeshEmpty;
    const double4 p = pack4[i];
    mpos[q] = p;
    const uint64_t k = keys[q];
    if (k == empty) {
        if (q == 0 || keys[q - 1] != empty) ms->n_in = (int32_t)q;
        mcell[q] = make_int4(0, 0, 0, 0);
        return;
    }
    int4 c;
    cell_of(p.x, p.y, p.z, g, c);                  // in range: checked by k_mesh_keys
    mcell[q] = c;
    if (q > 0 && keys[q - 1] == k) return;
    if (dense) {
        grid[k].x = (int32_t)q;
        return;
    }
    // the table holds at most n_in <= half its slots, so a free slot is always found
    int64_t h = slot_of(k, mask);
    for (int64_t probes = 0; probes <= mask; probes++) {
        const unsigned long long prev = atomicCAS(&tab[h].key, kMeshEmpty, k);
        if (prev == kMeshEmpty) {
            tab[h].start = (int32_t)q;
            return;
        }
        h = (h + 1) & mask;
    }
    atomicOr(&st->status, (int32_t)ST_CAP_MESH);   // unreachable at half load
}

// the last moonlet of every cell closes its range
__global__ void k_mesh_run_ends(const DevState *__restrict__ st, MeshState *ms,
                                const uint64_t *__restrict__ keys, int64_t n, MeshSlot *tab,
                                int64_t mask, int2 *grid, uint64_t dense_empty) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n || (st->status & kSkipMask)) return;
    const bool dense = ms->dense != 0;
    if (q == 0 && dense) {                         // the grid now holds this build's cells
        ms->grid_sparse = 1;
        ms->prev_n = (int32_t)n;
    }
    const uint64_t k = keys[q];
    if (k == (dense ? dense_empty : kMeshEmpty) || (q + 1 < n && keys[q + 1] == k)) return;
    if (dense) {
        grid[k].y = (int32_t)(q + 1);
        return;
    }
    int64_t h = slot_of(k, mask);
    for (int64_t probes = 0; probes <= mask; probes++) {
        if (tab[h].key == k) {
            tab[h].end = (int32_t)(q + 1);
            return;
        }
        h = (h + 1) & mask;
    }
}

// ------------------------------------------------------------------ gravity
// mu = G m and m in sorted order
__global__ void k_mesh_mu(const uint32_t *__restrict__ idx, const double *__restrict__ m,
                          double G, int64_t n, double4 *mpos, double *mmass) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q < n) {
        const double mi = m[idx[q]];
        mpos[q].w = G * mi;
        mmass[q] = mi;
    }
}

// a candidate for the three most massive: mass, input index, sorted position
struct Cand {
    double m;
    uint32_t i;
    int q;                     // -1: none
};
static_assert(sizeof(Cand) == 16, "top-three candidates take 16 bytes");

// a before b: larger mass, then smaller input index
__device__ __forceinline__ bool heavier(double ma, uint32_t ia, int qa, double mb, uint32_t ib,
                                        int qb) {
    if (qa < 0) return false;
    if (qb < 0) return true;
    return ma > mb || (ma == mb && ia < ib);
}

// The best three so far, heaviest first, as plain scalars (they stay in registers).
struct Top3 {
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    uint32_t i0 = 0u, i1 = 0u, i2 = 0u;
    int q0 = -1, q1 = -1, q2 = -1;

    __device__ __forceinline__ void insert(double m, uint32_t i, int q) {
        if (heavier(m, i, q, m0, i0, q0)) {
            m2 = m1; i2 = i1; q2 = q1;
            m1 = m0; i1 = i0; q1 = q0;
            m0 = m; i0 = i; q0 = q;
        } else if (heavier(m, i, q, m1, i1, q1)) {
            m2 = m1; i2 = i1; q2 = q1;
            m1 = m; i1 = i; q1 = q;
        } else if (heavier(m, i, q, m2, i2, q2)) {
            m2 = m; i2 = i; q2 = q;
        }
    }
    __device__ __forceinline__ void insert(const Cand &c) { insert(c.m, c.i, c.q); }
    __device__ __forceinline__ Cand get(int k) const {
        return k == 0 ? Cand{m0, i0, q0} : (k == 1 ? Cand{m1, i1, q1} : Cand{m2, i2, q2});
    }
    // merge lane (this ^ o)'s three
    __device__ __forceinline__ void merge_xor(int o) {
        const double a = __shfl_xor(m0, o), b = __shfl_xor(m1, o), c = __shfl_xor(m2, o);
        const uint32_t ia = (uint32_t)__shfl_xor((int)i0, o), ib = (uint32_t)__shfl_xor((int)i1, o),
                       ic = (uint32_t)__shfl_xor((int)i2, o);
        const int qa = __shfl_xor(q0, o), qb = __shfl_xor(q1, o), qc = __shfl_xor(q2, o);
        insert(a, ia, qa);
        insert(b, ib, qb);
        insert(c, ic, qc);
    }
};

// block-wide best three, valid in thread 0
__device__ __forceinline__ void block_top3(Top3 &t, Cand *lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t.merge_xor(o);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
        lds[3 * w] = t.get(0);
        lds[3 * w + 1] = t.get(1);
        lds[3 * w + 2] = t.get(2);
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int v = 1; v < (int)(blockDim.x / kWave); v++) {
            t.insert(lds[3 * v]);
            t.insert(lds[3 * v + 1]);
            t.insert(lds[3 * v + 2]);
        }
}

__global__ void __launch_bounds__(kMeshBlock)
k_mesh_top_part(const DevState *__restrict__ st, const double *__restrict__ mmass,
                const uint32_t *__restrict__ idx, int64_t n, Cand *part) {
    __shared__ Cand lds[3 * kMeshBlock / kWave];
    if (st->status & kSkipMask) return;
    Top3 t;
    // eight strided items per round, their loads issued together
    constexpr int kBatch = 8;
    const int64_t stride = (int64_t)gridDim.x * kMeshBlock;
    for (int64_t q0 = blockIdx.x * (int64_t)kMeshBlock + threadIdx.x; q0 < n;
         q0 += kBatch * stride) {
        double m[kBatch];
        uint32_t id[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; b++) {
            const int64_t q = q0 + b * stride;
            m[b] = q < n ? mmass[q] : 0.0;
            id[b] = q < n ? idx[q] : 0u;
        }
#pragma unroll
        for (int b = 0; b < kBatch; b++) {
            const int64_t q = q0 + b * stride;
            if (q < n) t.insert(m[b], id[b], (int)q);
        }
    }
    block_top3(t, lds);
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x] = t.get(0);
        part[3 * blockIdx.x + 1] = t.get(1);
        part[3 * blockIdx.x + 2] = t.get(2);
    }
}

// the three most massive, and gravity's all-pairs list: the moonlets out of the
// mesh (sorted positions n_in..n-1), then the three most massive that are in it
__global__ void __launch_bounds__(kMeshTopBlocks)
k_mesh_top_final(DevState *st, MeshState *ms, int64_t n, const Cand *__restrict__ part,
                 int32_t *big) {
    __shared__ Cand lds[3 * kMeshTopBlocks / kWave];
    __shared__ int s_nbig;
    if (st->status & kSkipMask) return;
    Top3 t;
    t.insert(part[3 * threadIdx.x]);
    t.insert(part[3 * threadIdx.x + 1]);
    t.insert(part[3 * threadIdx.x + 2]);
    block_top3(t, lds);
    const int n_in = ms->n_in;
    const int nover = (int)n - n_in;
    if (threadIdx.x == 0) {
        int ntop = 0, nbig = nover;
        // the three are heaviest first, the missing ones (q = -1) last
        const int top[3] = {t.q0, t.q1, t.q2};
        ntop = (t.q0 >= 0) + (t.q1 >= 0) + (t.q2 >= 0);
        for (int k = 0; k < 3; k++) ms->top[k] = top[k];
        ms->ntop = ntop;
        for (int k = 0; k < ntop; k++) nbig += top[k] < n_in;
        if (nbig > kMaxMeshBig) {
            atomicOr(&st->status, (int32_t)ST_CAP_MESH);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)nbig);
            nbig = 0;
        } else {
            int b = nover;
            for (int k = 0; k < ntop; k++)
                if (top[k] < n_in) big[b++] = top[k];
        }
        ms->nbig = nbig;
        s_nbig = nbig;
    }
    __syncthreads();
    if (s_nbig > 0)
        for (int k = threadIdx.x; k < nover; k += blockDim.x) big[k] = n_in + k;
}

// One thread per moonlet of the mesh (sorted order): its neighbours (not among the
// all-pairs moonlets) cell by cell, then the all-pairs moonlets.  The three most
// massive only count their neighbours here; their sums come from k_mesh_big_sum.
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_gravity(DevState *st, MeshState *ms, const MeshSlot *__restrict__ tab, int64_t mask,
               const int2 *__restrict__ grid,
               const double4 *__restrict__ mpos, const int4 *__restrict__ mcell,
               const uint32_t *__restrict__ idx, const int32_t *__restrict__ big,
               int count, double *__restrict__ ax, double *__restrict__ ay,
               double *__restrict__ az, unsigned long long *cnt_part) {
    __shared__ unsigned long long s_red[kMeshBlock / kWave];
    if (st->status & kSkipMask) {
        if (threadIdx.x == 0) cnt_part[blockIdx.x] = 0;
        return;
    }
    const int64_t q = blockIdx.x * (int64_t)kMeshBlock + threadIdx.x;
    const int n_in = ms->n_in, nbig = ms->nbig;
    const int t0 = ms->top[0], t1 = ms->top[1], t2 = ms->top[2];
    unsigned long long cnt = 0;
    const bool live = q < n_in;
    const CellIndex ci = cell_index(ms, grid, tab, mask);
    if (live) {
        const int4 c = mcell[q];
        const double4 p = mpos[q];
        const bool top = q == t0 || q == t1 || q == t2;
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int2 e = cell_range(ci, c.x + dx, c.y + dy, c.z + dz);
                    for (int r = e.x; r < e.y; r++) {
                        if (r == q) continue;
                        cnt++;
                        if (top || r == t0 || r == t1 || r == t2) continue;
                        add_pull(mpos[r], p.x, p.y, p.z, a0, a1, a2);
                    }
                }
        if (!top) {
            for (int k = 0; k < nbig; k++) {
                const int r = big[k];
                if (r != q) add_pull(mpos[r], p.x, p.y, p.z, a0, a1, a2);
            }
            const uint32_t i = idx[q];
            ax[i] = a0; ay[i] = a1; az[i] = a2;
        }
    }
    if (count) {
        const unsigned long long t = block_sum_u64(cnt, s_red);
        if (threadIdx.x == 0) cnt_part[blockIdx.x] = t;
    }
}

// all-pairs sums of the big moonlets: block (chunk, row) sums a chunk of sources
// for big moonlets row, row + kMeshBigRows, ...
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_big_sum(const DevState *__restrict__ st, const MeshState *__restrict__ ms,
               const double4 *__restrict__ mpos, const int32_t *__restrict__ big, int64_t n,
               double *part) {
    __shared__ double red[3][kMeshBlock / kWave];
    if (st->status & kSkipMask) return;
    const int nbig = ms->nbig;
    const int64_t per = (n + kMeshChunks - 1) / kMeshChunks;
    const int64_t j0 = blockIdx.x * per;
    const int64_t j1 = j0 + per < n ? j0 + per : n;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = blockIdx.y; k < nbig; k += gridDim.y) {
        const int b = big[k];
        const double4 p = mpos[b];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kMeshBlock)
            if (j != b) add_pull(mpos[j], p.x, p.y, p.z, a0, a1, a2);
        for (int o = 32; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o);
            a1 += __shfl_xor(a1, o);
            a2 += __shfl_xor(a2, o);
        }
        if (lane == 0) { red[0][w] = a0; red[1][w] = a1; red[2][w] = a2; }
        __syncthreads();
        if (threadIdx.x < 3) {
            double v = 0.0;
            for (int q = 0; q < kMeshBlock / kWave; q++) v += red[threadIdx.x][q];
            part[((int64_t)k * kMeshChunks + blockIdx.x) * 3 + threadIdx.x] = v;
        }
        __syncthreads();
    }
}

__global__ void k_mesh_big_final(const DevState *__restrict__ st,
                                 const MeshState *__restrict__ ms, const int32_t *__restrict__ big,
                                 const uint32_t *__restrict__ idx, const double *__restrict__ part,
                                 double *ax, double *ay, double *az) {
    if (st->status & kSkipMask) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ms->nbig) return;
    double a[3] = {0.0, 0.0, 0.0};
    for (int c = 0; c < kMeshChunks; c++)
        for (int d = 0; d < 3; d++) a[d] += part[((int64_t)k * kMeshChunks + c) * 3 + d];
    const uint32_t i = idx[big[k]];
    ax[i] = a[0]; ay[i] = a[1]; az[i] = a[2];
}

// ------------------------------------------------------------------ collisions
// velocities and radii in mesh order, from their packed records
__global__ void k_mesh_vel(const uint32_t *__restrict__ idx, const double4 *__restrict__ pack4,
                           int64_t n, double4 *mvel) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        mvel[q] = pack4[idx[q]];
}

__global__ void k_mesh_col_init(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) { st->npairs = 0; st->col_tests = 0; }
}

// one thread per moonlet of the mesh: its neighbours later in sorted order
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_collide(DevState *st, MeshState *ms, const MeshSlot *__restrict__ tab, int64_t mask,
               const int2 *__restrict__ grid,
               const double4 *__restrict__ mpos, const double4 *__restrict__ mvel,
               const int4 *__restrict__ mcell, const uint32_t *__restrict__ idx, double dt,
               int count, int64_t *out, int64_t cap, unsigned long long *cnt_part,
               unsigned long long *tests_part) {
    __shared__ unsigned long long s_red[kMeshBlock / kWave];
    if (st->status & kSkipMask) {
        if (threadIdx.x == 0) { cnt_part[blockIdx.x] = 0; tests_part[blockIdx.x] = 0; }
        return;
    }
    const int64_t q = blockIdx.x * (int64_t)kMeshBlock + threadIdx.x;
    const int n_in = ms->n_in;
    unsigned long long cnt = 0, tests = 0;
    const bool live = q < n_in;
    const CellIndex ci = cell_index(ms, grid, tab, mask);
    if (live) {
        const int4 c = mcell[q];
        const double4 p = mpos[q], v = mvel[q];
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int2 e = cell_range(ci, c.x + dx, c.y + dy, c.z + dz);
                    for (int r = e.x; r < e.y; r++) {
                        if (r == q) continue;
                        cnt++;
                        if (r < q) continue;
                        const double4 pr = mpos[r], vr = mvel[r];
                        tests++;
                        if (pair_test(p.x, p.y, p.z, v.x, v.y, v.z, v.w, pr.x, pr.y, pr.z, vr.x,
                                      vr.y, vr.z, vr.w, dt))
                            record(out, cap, (unsigned long long *)&st->npairs, idx[q], idx[r]);
                    }
                }
    }
    const unsigned long long tt = block_sum_u64(tests, s_red);
    const unsigned long long tc = block_sum_u64(cnt, s_red);
    if (threadIdx.x == 0) {
        tests_part[blockIdx.x] = tt;
        if (count) cnt_part[blockIdx.x] = tc;
    }
}

// the moonlets out of the mesh against every moonlet (each pair of two of them once)
__global__ void __launch_bounds__(kMeshBlock)
k_mesh_collide_out(DevState *st, const MeshState *__restrict__ ms,
                   const double4 *__restrict__ mpos, const double4 *__restrict__ mvel,
                   const uint32_t *__restrict__ idx, int64_t n, double dt, int64_t *out,
                   int64_t cap, unsigned long long *tests_part) {
    __shared__ unsigned long long s_red[kMeshBlock / kWave];
    const int64_t slot = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (threadIdx.x == 0) tests_part[slot] = 0;
    if (st->status & kSkipMask) return;
    const int n_in = ms->n_in;
    const int nover = (int)n - n_in;
    if (nover > kMaxMeshBig) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
            atomicOr(&st->status, (int32_t)ST_CAP_MESH);
            atomicMax((unsigned long long *)&st->required, (unsigned long long)nover);
        }
        return;
    }
    const int64_t per = (n + kMeshChunks - 1) / kMeshChunks;
    const int64_t j0 = blockIdx.x * per;
    const int64_t j1 = j0 + per < n ? j0 + per : n;
    unsigned long long tests = 0;
    for (int k = blockIdx.y; k < nover; k += gridDim.y) {
        const int b = n_in + k;
        const double4 p = mpos[b], v = mvel[b];
        for (int64_t j = j0 + threadIdx.x; j < j1; j += kMeshBlock) {
            if (j == b || (j >= n_in && j < b)) continue;
            const double4 pr = mpos[j], vr = mvel[j];
            tests++;
            if (pair_test(p.x, p.y, p.z, v.x, v.y, v.z, v.w, pr.x, pr.y, pr.z, vr.x, vr.y, vr.z,
                          vr.w, dt))
                record(out, cap, (unsigned long long *)&st->npairs, idx[b], idx[j]);
        }
    }
    const unsigned long long t = block_sum_u64(tests, s_red);
    if (threadIdx.x == 0) tests_part[slot] = t;
}

int grid_of(int64_t n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

hipError_t launch_mesh_build(const Workspace &ws, const double *x, const double *y,
                             const double *z, const double *R, int64_t n, const ncorp_params &prm,
                             bool first, hipStream_t s) {
    const int64_t mask = ws.mtab_n - 1;
    if (ws.clear_mesh) k_mesh_clear_state<<<1, 64, 0, s>>>(ws.mesh);
    if (first && prm.mesh_gamma <= 0.0 && prm.mesh_rmax <= 0.0)
        k_mesh_rmax<<<1024, 256, 0, s>>>(x, y, z, n, ws.mesh);
    k_mesh_begin<<<1, 64, 0, s>>>(ws.mesh, ws.st, n, prm.mesh_neighbours, prm.mesh_aspect,
                                  prm.mesh_rmax, prm.mesh_gamma,
                                  prm.mesh_min_side / prm.mesh_cells);
    k_mesh_unset<<<1024, 256, 0, s>>>(ws.mesh, ws.mkeys, ws.mgrid, ws.mgrid_n);
    // the box partials use the counter partials' buffer (free during a build)
    int32_t *box_part = reinterpret_cast<int32_t *>(ws.count_part);
    const int kblk = grid_of(n, 256);
    k_mesh_keys<<<kblk, 256, 0, s>>>(ws.st, ws.mesh, x, y, z, R, n, ws.mkeys, ws.midx,
                                     box_part, ws.pack4);
    k_mesh_box<<<1, 1024, 0, s>>>(box_part, kblk, ws.mesh, ws.mgrid_n);
    // dense grid: keys become grid indices below 2^gbits, all-ones in those bits when
    // empty, and the sort skips the digits above (an even number of passes, so that
    // the result lands where the full sort leaves it)
    int gbits = 1;
    while (gbits < 63 && (1ll << gbits) <= ws.mgrid_n) gbits++;
    const uint64_t dense_empty = (1ull << gbits) - 1ull;
    int keep = (gbits + 7) / 8;
    if ((8 - keep) % 2) keep++;
    k_mesh_clear_table<<<4096, 256, 0, s>>>(ws.mesh, ws.mtab, ws.mtab_n, ws.mgrid, ws.mgrid_n,
                                            ws.mkeys, n, dense_empty);
    // eight 8-bit passes (or `keep` of them) leave the result in mkeys / midx
    bool in_b = false;
    hipError_t e = launch_radix_sort(ws.mkeys, ws.midx, ws.mkeys_alt, ws.midx_alt, n, 64, ws.hist,
                                     &in_b, s, &ws.mesh->dense, keep);
    if (e != hipSuccess) return e;
    if (in_b) return hipErrorInvalidValue;
    k_mesh_runs<<<grid_of(n, 256), 256, 0, s>>>(ws.st, ws.mesh, ws.mkeys, ws.midx, ws.pack4, n,
                                                ws.mtab, mask, ws.mgrid, ws.mpos, ws.mcell,
                                                dense_empty);
    k_mesh_run_ends<<<grid_of(n, 256), 256, 0, s>>>(ws.st, ws.mesh, ws.mkeys, n, ws.mtab, mask,
                                                    ws.mgrid, dense_empty);
    return hipGetLastError();
}

hipError_t launch_mesh_gravity(const Workspace &ws, const double *m, double G, int64_t n,
                               bool count, double *ax, double *ay, double *az, hipStream_t s) {
    k_mesh_mu<<<grid_of(n, 256), 256, 0, s>>>(ws.midx, m, G, n, ws.mpos, ws.mmass);
    Cand *part = reinterpret_cast<Cand *>(ws.mtop_part);
    k_mesh_top_part<<<kMeshTopBlocks, kMeshBlock, 0, s>>>(ws.st, ws.mmass, ws.midx, n, part);
    k_mesh_top_final<<<1, kMeshTopBlocks, 0, s>>>(ws.st, ws.mesh, n, part, ws.mbig);
    const int nblk = grid_of(n, kMeshBlock);
    k_mesh_gravity<<<nblk, kMeshBlock, 0, s>>>(ws.st, ws.mesh, ws.mtab, ws.mtab_n - 1, ws.mgrid,
                                               ws.mpos,
                                               ws.mcell, ws.midx, ws.mbig, count ? 1 : 0, ax, ay,
                                               az, ws.count_part);
    if (count) k_mesh_count_done<<<1, 1024, 0, s>>>(ws.count_part, nblk, ws.mesh);
    k_mesh_big_sum<<<dim3(kMeshChunks, kMeshBigRows), kMeshBlock, 0, s>>>(ws.st, ws.mesh,
                                                                         ws.mpos, ws.mbig, n,
                                                                         ws.mbig_part);
    k_mesh_big_final<<<kMaxMeshBig / 256, 256, 0, s>>>(ws.st, ws.mesh, ws.mbig, ws.midx,
                                                      ws.mbig_part, ax, ay, az);
    return hipGetLastError();
}

hipError_t launch_mesh_collide(const Workspace &ws, const double *vx, const double *vy,
                               const double *vz, const double *R, int64_t n, double dt,
                               bool count, hipStream_t s) {
    hipError_t e0 = launch_pack_vr(ws, vx, vy, vz, R, n, s);
    if (e0 != hipSuccess) return e0;
    k_mesh_vel<<<grid_of(n, 256), 256, 0, s>>>(ws.midx, ws.pack4, n, ws.mvel);
    k_mesh_col_init<<<1, 64, 0, s>>>(ws.st);
    // partials: neighbour counts [0, nblk), tests [nblk, 2 nblk), tests of the moonlets
    // out of the mesh [2 nblk, 2 nblk + kMeshChunks * kMeshBigRows)
    const int nblk = grid_of(n, kMeshBlock);
    unsigned long long *cnt = ws.count_part, *tst = ws.count_part + nblk;
    k_mesh_collide<<<nblk, kMeshBlock, 0, s>>>(ws.st, ws.mesh, ws.mtab, ws.mtab_n - 1, ws.mgrid,
                                               ws.mpos,
                                               ws.mvel, ws.mcell, ws.midx, dt, count ? 1 : 0,
                                               ws.pairs_tmp, ws.pair_cap, cnt, tst);
    k_mesh_collide_out<<<dim3(kMeshChunks, kMeshBigRows), kMeshBlock, 0, s>>>(
        ws.st, ws.mesh, ws.mpos, ws.mvel, ws.midx, n, dt, ws.pairs_tmp, ws.pair_cap,
        tst + nblk);
    if (count) k_mesh_count_done<<<1, 1024, 0, s>>>(cnt, nblk, ws.mesh);
    return launch_sum_u64(tst, nblk + kMeshChunks * kMeshBigRows,
                          (unsigned long long *)&ws.st->col_tests, true, s);
}

}  // namespace ncorp

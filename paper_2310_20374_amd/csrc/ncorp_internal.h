// Internal definitions shared by the HIP translation units of libncorp.
// Device code targets gfx950 (wave64).  All device memory comes from the caller's
// workspace; `Workspace` records where each array lives inside it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ncorp.h"

namespace ncorp {

constexpr int kMaxDepth = 21;          // 63-bit keys: 21 levels of 3 bits
constexpr int kMaxP = 6;
constexpr int kWave = 64;
// The hardware deals the workgroups of a launch to the 8 XCDs in turn (workgroup b
// runs on XCD b mod 8), and each XCD has its own L2.
constexpr int kXcds = 8;
// the climbs' per-XCD leaf counters: one counter per 128-byte line
constexpr int kCtrStride = 32;

// ---------------------------------------------------------------- tensor sizes
// Symmetric tensors are stored per order n as the (n+1)(n+2)/2 components
// a = (ax, ay, az), |a| = n, ordered by ax descending then ay descending.
__host__ __device__ constexpr int tri(int k) { return k * (k + 1) / 2; }
__host__ __device__ constexpr int ncomp(int n) { return (n + 1) * (n + 2) / 2; }
// components of all orders below n
__host__ __device__ constexpr int off_order(int n) { return n * (n + 1) * (n + 2) / 6; }
// index of multi-index (a, b, c) among all orders
__host__ __device__ constexpr int sidx(int a, int b, int c) {
    return off_order(a + b + c) + tri(b + c) + c;
}
// multipoles: orders 0 and 2..p-1 (order 1 vanishes at the centre of mass)
__host__ __device__ constexpr int n_mult(int p) {
    return p <= 0 ? 0 : (p == 1 ? 1 : off_order(p) - 3);
}
__host__ __device__ constexpr int midx(int a, int b, int c) {
    return (a + b + c) == 0 ? 0 : sidx(a, b, c) - 3;
}
// interaction tensors C^(m), m = 1..p
__host__ __device__ constexpr int n_local(int p) { return p <= 0 ? 0 : off_order(p + 1) - 1; }
__host__ __device__ constexpr int cidx(int a, int b, int c) { return sidx(a, b, c) - 1; }

// ---------------------------------------------------------------- status word
enum StatusBits : int32_t {
    ST_CAP_CELLS = 1, ST_CAP_QUEUE = 2, ST_CAP_M2L = 4, ST_CAP_P2P = 8,
    ST_CAP_PAIRS = 16, ST_NONFINITE = 32, ST_CAP_LISTS = 64, ST_WALK_STALL = 128,
    ST_BAD_ITEM = 256, ST_BAD_OFFSETS = 512, ST_MESH_RANGE = 1024, ST_CAP_MESH = 2048
};
// Any of these leaves the tree or the interaction lists incomplete: later passes
// then do nothing rather than follow indices that were never written.
// persistent walk: waves, and list slots a wave reserves at a time (the plain
// cell-pair lists carry up to kWalkWaves * kListChunk slots of gaps)
// items per tile of the radix sort's passes (the workspace sizes its histograms by it)
constexpr int kSortTileItems = 2048;
// bucket sort of a plain tree build: buckets of kBucketMean moonlets on average, a
// bucket of up to kBucketLDS sorted in LDS by one block (larger ones in such chunks,
// merged); at most kMaxBuckets buckets (more moonlets: the radix sort); the count and
// scatter passes take kBucketTile moonlets per block
constexpr int kBucketMean = 1792;
constexpr int kBucketLDS = 4096;
constexpr int kMaxBuckets = 3200;
constexpr int kBucketTile = 2048;
// the previous build's keys at every kSubStride-th rank split each bucket again
constexpr int kSubStride = 8;
constexpr int kWalkBlock = 256;
// persistent blocks: the gravity walk runs 1024 waves, the collision walk (less
// work per item) 512; more only adds contention on the queue counters
constexpr int kWalkGridGravity = 256;
constexpr int kWalkGridCollide = 128;
constexpr int kWalkWaves = kWalkGridGravity * kWalkBlock / kWave;
constexpr int kWalkWavesMax = 2048;       // the largest walk_waves
// persistent waves of the gravity walk under these parameters
inline int walk_waves(const ncorp_params &p) { return p.walk_waves > 0 ? p.walk_waves : kWalkWaves; }
constexpr int kListChunk = 256;
// the walk's tail shares a 64-bit word with the processed count (32 bits each); an
// item pushes at most 36 children, so a queue of this many slots keeps the tail
// below 2^32 even when it overflows
constexpr int64_t kMaxQueue = 100000000;
// workspace bytes per colliding-pair slot: two key buffers, contact time, state
constexpr int64_t kPairBytes = 8 + 8 + 8 + 4;

// per-target interaction lists: default and largest slot counts (a consumer
// sorts a whole list in LDS)
constexpr int kDefaultM2LPerCell = 2048;
constexpr int kDefaultP2PPerLeaf = 4096;
constexpr int kMaxPerTarget = 8192;
// lists up to these lengths are sorted in LDS by their consumer; longer ones (the
// walk records them) by a pre-pass of kSortLongBlocks single-wave blocks per kind
constexpr int kM2LListLDS = 512;
constexpr int kP2PListLDS = kWave;
constexpr int kSortLongBlocks = 1024;
// direct sums of a leaf with a long source list are split over kLongSlots waves
// (kLongGrid extra four-wave blocks); their partial sums meet in p2p_part
constexpr int kLongSlots = 8;
constexpr int kLongGrid = 2048;

constexpr int32_t kSkipMask = ST_CAP_CELLS | ST_CAP_QUEUE | ST_CAP_M2L | ST_CAP_P2P |
                              ST_CAP_LISTS | ST_WALK_STALL | ST_BAD_ITEM | ST_BAD_OFFSETS |
                              ST_MESH_RANGE | ST_CAP_MESH;

// independent disks of one batched call (a forest with one root per non-empty disk)
constexpr int kMaxDisks = NCORP_MAX_DISKS;

// Device-side counters of one tree / walk, kept in the workspace.
struct DevState {
    int32_t status;            // StatusBits, latched
    int32_t pad0;
    int64_t required;          // size that would have sufficed for an overflow
    // tree
    int32_t ncells, nleaves, maxlevel, pad1;
    int32_t level_count[kMaxDepth + 2];
    int32_t level_off[kMaxDepth + 3];
    double L;                  // root half-width (of disk 0 in a batched call)
    double max_abs;            // max |coordinate| (bit pattern max for >= 0 doubles)
    int32_t ndisks, nroots;    // disks of the call; level-0 cells (non-empty disks)
    // gravity walk
    int32_t nm2l, np2p;        // unordered cell pairs (exact counts)
    int32_t m2l_slots, p2p_slots;  // list slots reserved (entries plus (-1,-1) gaps)
    int32_t m2l_maxlist, p2p_maxlist;  // longest per-target lists (timing runs only)
    int32_t nlong_m2l, nlong_p2p;      // lists longer than their consumer's LDS sort
    int64_t visited;
    // collision walk
    int32_t ncand, cand_slots;
    int64_t col_tests;
    int64_t npairs;            // colliding pairs found (may exceed capacity)
    int64_t pair_cursor;       // pairs already written by earlier steps of ncorp_step
    int64_t p2p_inter;         // directed moonlet pairs (i != j) of the direct sums
    // load balance of the last gravity evaluation (timing runs only): busy cycles of
    // the gravity walk's waves (sum and max over the persistent waves) and the most
    // source moonlets any leaf's direct sums take
    int64_t walk_busy_sum, walk_busy_max;
    int64_t p2p_src_max;
    // collisions: the largest R + dt |v| of any moonlet (bit pattern of a double >= 0)
    unsigned long long reach_max;
    // bucket sort: the splitters the last bucket sort left for the next one are valid
    // (bs_valid) for bs_n moonlets under root half-width bs_L (kept by the reset of a
    // fresh build); the last sort took its buckets from them (bs_prev_used) and sorted
    // bs_spill buckets too large for one LDS batch by merging
    double bs_L;
    int32_t bs_valid, bs_n;
    int32_t bs_prev_used, bs_spill;
    // which of the two sub-boundary buffers the last sort wrote (kept like bs_valid),
    // and which this sort reads
    int32_t bs_sub_wr, bs_sub_rd;
};

// a bucket boundary of the bucket sort: the (key, input index) pair that starts it
struct SplitKey {
    uint64_t k;
    uint32_t i, pad;
};

// ---------------------------------------------------------------- mesh module
// Moonlets that interact with every other one in the mesh module: those too large
// for the mesh (2R > gamma) and, for gravity, the three most massive.
constexpr int kMaxMeshBig = 1024;
constexpr int kMeshCellLimit = 1 << 20;  // |cell coordinate| bound (21-bit Morton axes)
// a slot of the mesh's cell table: the Morton key of an occupied cell and the
// range [start, end) of its moonlets in sorted order
struct MeshSlot {
    unsigned long long key;            // kMeshEmpty: free
    int32_t start, end;
};
constexpr unsigned long long kMeshEmpty = ~0ull;
// State of the mesh across builds (lives in the workspace, cleared when a new
// workspace buffer is bound).
struct MeshState {
    double gamma;                      // mesh size of the current mesh
    double rmax2;                      // max |r|^2 at the first mesh (R_max of Eq. 4)
    unsigned long long nbr_sum;        // (moonlet, neighbour) pairs counted on it
    int32_t n_in;                      // moonlets in the mesh: the sorted prefix
    int32_t stamp;                     // build counter
    int32_t init;                      // gamma has been set
    int32_t measured;                  // nbr_sum counted on the current mesh
    int32_t ntop;                      // the three most massive (sorted positions)
    int32_t top[3];
    int32_t nbig;                      // gravity's all-pairs list (mesh_big)
    // the box of occupied cells; dense = its cells are indexed directly (mgrid)
    // instead of through the hash table
    int32_t box_x0, box_y0, box_z0, box_dx, box_dy, box_dz;
    int32_t dense;
    // grid_sparse: the last build was dense and completed, so the whole grid buffer is
    // zero except at the first prev_n sorted keys (its cells); grid_zero: this build
    // found it so and cleared those cells
    int32_t grid_sparse, prev_n, grid_zero;
    int32_t pad[3];
};

// Work-queue state of a persistent walk; each counter on its own 128-byte line.
struct WalkQueue {
    uint64_t head;             // next slot to claim
    uint64_t pad0[15];
    uint64_t tp;               // next slot to reserve (high 32 bits) and items
                               // processed (low 32 bits), updated by one atomic
    uint64_t pad1[15];
    uint64_t pad2[16];
    uint32_t epoch;            // tag of the last walk's items (advanced on the device)
    uint32_t epoch_next;       // tag of this walk's items (written by its init pass)
    uint32_t pad3[30];
};

// What the walk reads of a cell, one 64-byte line: centre, critical radius,
// moonlet count, first child, number of children (0 for a leaf), first leaf and
// number of leaves below it.
struct alignas(64) WCell {
    double x, y, z, rcrit;
    int32_t count, child, nchild, entry, nent, first, pad[2];
};

// Waves of a multi-wave block that work independently synchronise their own LDS
// traffic only: a wave's LDS operations complete in issue order, so it suffices to
// keep the compiler from moving LDS accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sorts a per-target list list[0..len) ascending, in place in global memory (its
// values are distinct).  Called by a whole single-wave block; scratch is LDS of at
// least round_up(len, 4) ints, 16-byte aligned.  Ends with a block barrier, so the
// wave's later loads see the sorted list.
__device__ __forceinline__ void sort_target_list(int32_t *list, int len, int32_t *scratch) {
    const int lane = threadIdx.x;
    const int len4 = (len + 3) & ~3;
    for (int i = lane; i < len4; i += kWave) scratch[i] = i < len ? list[i] : 0x7fffffff;
    __syncthreads();
    const int4 *s4 = reinterpret_cast<const int4 *>(scratch);
    for (int i = lane; i < len; i += kWave) {
        const int v = scratch[i];
        int r = 0;
        #pragma unroll 8
        for (int j = 0; j < len4 / 4; j++) {
            const int4 t = s4[j];
            r += (t.x < v) + (t.y < v) + (t.z < v) + (t.w < v);
        }
        list[r] = v;
    }
    __syncthreads();
}

// ---------------------------------------------------------------- workspace
struct Workspace {
    char *base = nullptr;
    int64_t bytes = 0;
    int64_t n_max = 0, cell_cap = 0, m2l_cap = 0, p2p_cap = 0, queue_cap = 0;
    int64_t leaf_cap = 0, pair_cap = 0;
    int m2l_stride = 0, p2p_stride = 0;               // slots per target list
    int p = 0, nm = 0, nl = 0;
    // per moonlet (tree order unless noted)
    uint64_t *keys = nullptr, *keys_alt = nullptr;
    uint32_t *idx = nullptr, *idx_alt = nullptr;      // tree position -> input index
    uint32_t *code = nullptr;                         // tree-build per-moonlet code
    double *xs = nullptr, *ys = nullptr, *zs = nullptr, *mus = nullptr;
    double *vxs = nullptr, *vys = nullptr, *vzs = nullptr, *rads = nullptr;
    // packed 32-byte records in input order, staging for the gathers into tree or
    // mesh order: (x, y, z, 0) from the key passes, (vx, vy, vz, R) before a
    // collision search
    double4 *pack4 = nullptr;
    double4 *pcol = nullptr;                          // x, y, z, R + dt |v| (collisions)
    double4 *vcol = nullptr;                          // vx, vy, vz, R (tree order, collisions)
    double4 *cbox = nullptr;                          // per leaf: box low corner + largest
                                                      // R + dt |v|, box high corner
    double *acc = nullptr;                            // 3 x n, input order (step)
    double *acc_s = nullptr;                          // 3 x n, tree order (direct sums)
    // leaves in moonlet order ("entries")
    int32_t *ent_start = nullptr;                     // first moonlet
    uint32_t *ent_code = nullptr;                     // dv | L << 8
    int32_t *ent_cell = nullptr;                      // cell index of the leaf
    // cells, breadth-first
    int32_t *c_level = nullptr, *c_first = nullptr, *c_count = nullptr;
    int32_t *c_child = nullptr, *c_nchild = nullptr, *c_parent = nullptr;
    int32_t *c_entry = nullptr;                       // first leaf (entry index)
    int32_t *c_nent = nullptr;                        // number of leaves below
    uint64_t *c_prefix = nullptr;
    int32_t *c_arrive = nullptr;                      // climb counters
    int32_t *climb_next = nullptr;   // climbs: next leaf of each XCD slice (kXcds x 32)
    double4 *gcell = nullptr;                         // s_x, s_y, s_z, r_crit
    double *c_mass = nullptr, *c_rmax = nullptr, *c_theta = nullptr;
    double *mult = nullptr;                           // cell_cap x nm (FP64)
    float *mult32 = nullptr;                          // cell_cap x nm (FP32)
    double *local = nullptr;                          // cell_cap x nl (C after walk)
    double *cleaf = nullptr;                          // n_max x nl (C at each leaf)
    double4 *ccell = nullptr;                         // sbar, r_crit (collisions)
    WCell *wg = nullptr, *wc = nullptr;               // walk records: gravity, collisions
    double *c_crmax = nullptr;
    // walks
    uint64_t *queue = nullptr;
    WalkQueue *wq = nullptr;
    int2 *m2l = nullptr, *p2p = nullptr;              // unordered cell pairs
    int2 *cand = nullptr;                             // collision candidate cell pairs
    // per-target lists written by the gravity walk (unordered; consumers sort)
    int32_t *m2l_cnt = nullptr, *m2l_seg = nullptr;   // by target cell, m2l_stride slots
    int32_t *p2p_cnt = nullptr, *p2p_seg = nullptr;   // by target leaf, p2p_stride slots
    int32_t *long_m2l = nullptr, *long_p2p = nullptr; // targets of over-long lists
    double *p2p_part = nullptr;                       // kLongSlots x 3 x n partial sums
    int32_t *cnt_a = nullptr;                         // tree-build level counters
    int64_t *pairs_tmp = nullptr;                     // colliding pairs (i<<32|j)
    int64_t *pairs_alt = nullptr;
    // collision resolution: contact time and state of each pair, best pair and
    // "already collided" flag of each moonlet (input order)
    double *pair_dt = nullptr;
    int32_t *pair_flag = nullptr;
    int32_t *mbest = nullptr, *mmatch = nullptr;
    int32_t *cand_blk = nullptr;                      // per-block candidate counts
    // scratch for scans and sorts
    int32_t *scan_part = nullptr;                     // block partials
    uint32_t *hist = nullptr;                         // radix histograms
    // bucket sort: this build's bucket boundaries, those for the next build (the keys
    // at ranks j kBucketMean of this one), the finer boundaries (keys at ranks
    // k kSubStride, one buffer read while the other is written), moonlets per
    // (bucket, tile) (bucket-major,
    // then their exclusive prefix over the tiles), moonlets per bucket, bucket starts
    // (n_buckets + 1); sort_prev: a bucket sort on this binding wrote bs_prev (the
    // device still checks n and the root cube)
    SplitKey *bs_split = nullptr, *bs_prev = nullptr;
    SplitKey *bs_sub[2] = {nullptr, nullptr};         // keys at ranks k kSubStride
    uint32_t *bs_cm = nullptr, *bs_total = nullptr, *bs_off = nullptr;
    uint32_t *bs_done = nullptr;                      // bucket sorted by the fast pass
    bool sort_prev = false;
    // batched calls: disk of each moonlet (input order; the sort keeps disks
    // contiguous, so it is also the disk of each tree position), per-disk max
    // |coordinate| and root half-width
    uint16_t *seg = nullptr;
    unsigned long long *disk_max = nullptr;
    double *disk_L = nullptr;
    int32_t *disk_root = nullptr;                     // level-0 cell of each disk
    int ndisks = 1;                                   // host copy; 1 = plain call
    // mesh module (present when a method uses it): moonlets sorted by the Morton
    // key of their cell (those out of the mesh last), and an open-addressing table
    // of the occupied cells (a power of two >= 2 n_max slots)
    MeshState *mesh = nullptr;
    MeshSlot *mtab = nullptr;
    int64_t mtab_n = 0;
    int2 *mgrid = nullptr;                            // dense cell index of the box
    int64_t mgrid_n = 0;
    uint64_t *mkeys = nullptr, *mkeys_alt = nullptr;
    uint32_t *midx = nullptr, *midx_alt = nullptr;   // sorted position -> input index
    double4 *mpos = nullptr;                          // x, y, z, mu (sorted)
    int4 *mcell = nullptr;                            // cell coordinates (sorted)
    double4 *mvel = nullptr;                          // vx, vy, vz, R (sorted)
    int32_t *mbig = nullptr;                          // kMaxMeshBig sorted positions
    double *mmass = nullptr;                          // masses (sorted)
    void *mtop_part = nullptr;                        // per-block top-three candidates
    double *mbig_part = nullptr;                      // partial sums of the big ones
    unsigned long long *count_part = nullptr;         // per-block counter partials
    int64_t count_part_n = 0;
    DevState *st = nullptr;
    bool timing = false;                              // phase timing on: load-balance counters
    bool clear_queue = false;                         // new buffer: clear before next walk
    bool clear_mesh = false;                          // new buffer: clear the mesh state
    // the climbs' arrival and leaf counters are zero: the last tree build's cell-range
    // pass cleared them and no climb has run since
    bool arrive_clean = false;
};

// Layout of the workspace for given capacities; with base == nullptr only the
// size is computed.
int64_t layout_workspace(Workspace &ws, const ncorp_params &prm, int64_t n_max,
                         int64_t pair_cap);

// ---------------------------------------------------------------- launchers
// (each returns hipSuccess or the first launch error)
hipError_t launch_reset_state(const Workspace &ws, hipStream_t s);
hipError_t launch_gather_scaled(const Workspace &ws, const double *src, double scale,
                                double *dst, int64_t n, hipStream_t s);
// disk_off: n_disks + 1 device offsets of a batched call (nullptr for a plain call);
// m: masses (input order) to pack as G m beside the positions, or nullptr;
// max_ready (plain calls): the step's drift has already formed max |coordinate|
hipError_t launch_keys(const Workspace &ws, const double *x, const double *y,
                       const double *z, int64_t n, double root_half_width,
                       const int64_t *disk_off, const double *m, double G, hipStream_t s,
                       bool max_ready = false);
hipError_t launch_sort(const Workspace &ws, int64_t n, hipStream_t s);
// plain builds of up to kMaxBuckets buckets use the bucket sort (launch_keys then
// writes where it starts)
bool bucket_sort_applies(const Workspace &ws, int64_t n);
hipError_t launch_bucket_sort(const Workspace &ws, int64_t n, hipStream_t s);
// with_mus: the keys packed G m, which lands in ws.mus too
hipError_t launch_gather_pos(const Workspace &ws, int64_t n, bool with_mus, hipStream_t s);
hipError_t launch_gather(const Workspace &ws, const double *src, double *dst, int64_t n,
                         hipStream_t s);
// velocities and radii into tree order, one pass
hipError_t launch_pack_vr(const Workspace &ws, const double *vx, const double *vy,
                          const double *vz, const double *R, int64_t n, hipStream_t s);
hipError_t launch_gather_vr(const Workspace &ws, bool packed, const double *vx, const double *vy,
                            const double *vz, const double *R, int64_t n, hipStream_t s);
hipError_t launch_build_tree(const Workspace &ws, int64_t n, int leaf_size, hipStream_t s);

// reset: clear the arrival and leaf counters first (not needed right after a build);
// rcrit: then the opening angles and critical radii (a gravity walk's init pass can
// do them instead)
hipError_t launch_gravity_climb(const Workspace &ws, int64_t n, const ncorp_params &prm,
                                hipStream_t s, bool reset = true, bool rcrit = true);
hipError_t launch_collision_climb(const Workspace &ws, int64_t n, double dt, hipStream_t s,
                                  bool reset = true);

// walk: mode 0 gravity (M2L + P2P lists), 1 collisions (candidate list in p2p)
// rcrit_prm (gravity walk): its init pass also forms the opening angles and critical
// radii the climb left out
hipError_t launch_walk(Workspace &ws, int mode, int ncs, int ncc_pre, int ncc_post, int waves,
                       hipStream_t s, const ncorp_params *rcrit_prm = nullptr);
hipError_t launch_count_interactions(const Workspace &ws, hipStream_t s);
// sorts, in place, the per-target lists longer than the consumers sort in LDS
hipError_t launch_sort_long_lists(const Workspace &ws, hipStream_t s);

hipError_t launch_m2l(const Workspace &ws, int p, int precision, hipStream_t s);
hipError_t launch_l2l(const Workspace &ws, int p, hipStream_t s);
hipError_t launch_p2p(const Workspace &ws, int64_t n, int precision, int tile, int tmax,
                      hipStream_t s);
// acc4 non-null: the accelerations as one (ax, ay, az, 0) record per moonlet in
// input order instead of the three arrays (one scattered record, not three words)
hipError_t launch_l2p(const Workspace &ws, int64_t n, int p, double *ax, double *ay, double *az,
                      hipStream_t s, double4 *acc4 = nullptr);
// brute-force module (every pair): accelerations by input index; colliding pairs
hipError_t launch_brute_gravity(const Workspace &ws, int64_t n, double *ax, double *ay,
                                double *az, hipStream_t s);
hipError_t launch_brute_collide(const Workspace &ws, int64_t n, double dt, hipStream_t s);
// clears the pair and test counters before a collision search
hipError_t launch_collide_reset(const Workspace &ws, hipStream_t s);
// standard tree code (Alg. 1), collision form: colliding pairs into pairs_tmp
hipError_t launch_standard_tree_collide(const Workspace &ws, int64_t n, int ncb_pre,
                                        int ncb_post, double dt, hipStream_t s);
// standard tree code (Alg. 1): accelerations of all moonlets, input order
hipError_t launch_standard_tree(const Workspace &ws, int64_t n, int p, int ncb_pre, int ncb_post,
                                double *ax, double *ay, double *az, hipStream_t s);
// blocks of the tree's pair tests (one wave each): each leaves its number of examined
// pairs in ws.count_part (at least 33 920 entries at any n), which the pair ranking that
// follows adds to st->col_tests
constexpr int kCollideGrid = 32768;
hipError_t launch_collide_pairs(const Workspace &ws, int64_t n, double dt, bool boxes,
                                hipStream_t s);
hipError_t launch_leaf_boxes(const Workspace &ws, int64_t n, double dt, hipStream_t s);
// collision candidates from the gravity walk's lists of the same tree (in place of
// the collision walk)
hipError_t launch_candidates_from_lists(const Workspace &ws, hipStream_t s);
// tests_part: n_part per-block counts of examined pairs to add to st->col_tests (the
// tree's pair tests leave them), or nullptr
hipError_t launch_emit_pairs(const Workspace &ws, int64_t *pairs, int64_t cap,
                             int64_t *n_pairs_dev, int triple, int step, int64_t *cursor,
                             const unsigned long long *tests_part, int n_part, hipStream_t s);
// sorts the pairs found, resolves them (caller arrays in input order, updated in
// place) and writes the resolved ones as (step, i, j) triples
hipError_t launch_resolve(const Workspace &ws, double *x, double *y, double *z, double *vx,
                          double *vy, double *vz, const double *m, const double *R, double dt,
                          double f, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev, int step,
                          int64_t *cursor, const unsigned long long *tests_part, int n_part,
                          hipStream_t s);

// dst (+)= sum of n per-block partials (one block, fixed order)
hipError_t launch_sum_u64(const unsigned long long *part, int64_t n, unsigned long long *dst,
                          bool add, hipStream_t s);
// mesh module (Sect. 3.3)
hipError_t launch_radix_sort(uint64_t *ka, uint32_t *va, uint64_t *kb, uint32_t *vb, int64_t n,
                             int bits, uint32_t *hist, bool *in_b, hipStream_t s,
                             const int32_t *skip = nullptr, int skip_from = 0);
hipError_t launch_mesh_build(const Workspace &ws, const double *x, const double *y,
                             const double *z, const double *R, int64_t n, const ncorp_params &prm,
                             bool first, hipStream_t s);
hipError_t launch_mesh_gravity(const Workspace &ws, const double *m, double G, int64_t n,
                               bool count, double *ax, double *ay, double *az, hipStream_t s);
hipError_t launch_mesh_collide(const Workspace &ws, const double *vx, const double *vy,
                               const double *vz, const double *R, int64_t n, double dt,
                               bool count, hipStream_t s);

// what the kick adds besides the mutual gravity: G M_c, G M_c R^2 J2, and the
// distant body (G M_sun, its position, a^2, a^3); zero factors switch terms off
struct CentralBody {
    double GM, GMR2J2, GMsun, sx, sy, sz, a2, a3;
};
// acc4 non-null: the accelerations as (ax, ay, az, 0) records (ax .. az unused)
hipError_t launch_kick(double *vx, double *vy, double *vz, const double *ax,
                       const double *ay, const double *az, const double *x,
                       const double *y, const double *z, int64_t n, double h,
                       const CentralBody &b, const double *R, double4 *pack, hipStream_t s,
                       const double4 *acc4 = nullptr);
// st non-null: also max |coordinate| of the new positions into st->max_abs, as the key
// pass of a plain build forms it (the previous build's cell-range pass cleared it)
hipError_t launch_drift(double *x, double *y, double *z, const double *vx,
                        const double *vy, const double *vz, int64_t n, double dt,
                        hipStream_t s, DevState *st = nullptr);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_i64(int64_t *p, int64_t v, int64_t n, hipStream_t s);

// device-wide exclusive scan of n_dev[0] int32 values (n_cap an upper bound);
// writes total to *total_dev (may alias out[n]).
hipError_t launch_scan(const int32_t *in, int32_t *out, const int32_t *n_dev, int64_t n_cap,
                       int32_t *partials, int32_t *total_dev, hipStream_t s);

}  // namespace ncorp

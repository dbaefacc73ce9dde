/*
 * ncorp.h -- C ABI of libncorp, the MI355X (gfx950) falcON tree step.
 *
 * The library implements the falcON-style O(N) tree step of NcorpiON
 * (Couturier, Quillen & Nakajima): Hilbert-key sort and octree build
 * (Sect. 3.4.1, Sect. 3.4.6), upward pass with Cartesian multipole moments up to
 * order 6 (Eq. 20, App. C), the dual tree walk (Alg. 2) with interaction tensors
 * (Eq. 25) and direct sums, the downward shift (Eq. 26), the same walk reused
 * for collision search (Sect. 3.1 Eqs. 1-2, Eqs. 7-9), and a kick-drift-kick
 * leapfrog around a central mass (Sect. 4.1, App. B.1).
 *
 * Conventions for every entry point:
 *  - Memory.  Every array argument is a DEVICE pointer owned by the caller.  The
 *    library never allocates device memory: all scratch space lives in the
 *    caller's workspace (ncorp_workspace_bytes).  Arrays are plain
 *    structure-of-arrays, FP64 unless noted, indexed by the caller's (input)
 *    moonlet index.
 *  - Streams.  `stream` is a hipStream_t passed as void* (NULL = default
 *    stream).  Calls only enqueue work and return; nothing waits for the GPU
 *    except ncorp_get_status, ncorp_tree_info and ncorp_export_host.
 *  - Errors.  Argument errors are detected on the host and returned at once
 *    (NCORP_E_INVALID, nothing enqueued).  Conditions only the GPU can see
 *    (a capacity exceeded, a non-finite position) are latched in a status word
 *    inside the workspace and reported by ncorp_get_status; outputs of such a
 *    call are then incomplete and must be discarded.
 *  - A context is not thread-safe and must not be used on two streams at once.
 *    Workspace contents persist between calls: ncorp_gravity and ncorp_collide
 *    use the tree of the last ncorp_build_tree on the same context.
 */
#ifndef NCORP_H
#define NCORP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NCORP_OK = 0,
    NCORP_E_INVALID = -1,      /* bad argument (host-side check) */
    NCORP_E_CAPACITY = -2,     /* a device list overflowed; see required size */
    NCORP_E_HIP = -3,          /* a HIP runtime call failed */
    NCORP_E_UNSUPPORTED = -4,  /* valid request this build does not provide */
    NCORP_E_NONFINITE = -5     /* a position was NaN or infinite */
} ncorp_status;

typedef enum {
    NCORP_FP64 = 0,            /* every floating-point step in FP64 */
    NCORP_FP32_BULK = 1        /* direct sums and interaction tensors in FP32 with
                                  compensated accumulation; positions, offsets,
                                  climbs, shifts and the integrator in FP64 */
} ncorp_precision;

/* Parameters of the method.  Defaults: ncorp_params_default. */
typedef struct {
    double G;                  /* gravitational constant (paper default 4 pi^2, App. B.1) */
    double M_central;          /* central mass, not part of the tree (Sect. 3.4.3) */
    int p;                     /* expansion order 0..6 (Sect. 3.4.3); 0 = no mutual gravity */
    double theta_min;          /* opening angle of the root cell, 0 < theta_min < 1 */
    int theta_mode;            /* 0: mass-dependent theta(M) (Sect. 3.4.2, Dehnen's
                                  relation); 1: constant theta = theta_min */
    int leaf_size;             /* s: cells with <= s moonlets are leaves (Sect. 3.4.1) */
    int ncs, ncc_pre, ncc_post;               /* gravity walk thresholds (Alg. 2) */
    int ncs_col, ncc_pre_col, ncc_post_col;   /* collision walk thresholds (Alg. 2) */
    int precision;             /* ncorp_precision */
    double root_half_width;    /* 0 = smallest power of two above every |coordinate| */
    /* capacities of device lists; 0 = automatic from n_max and leaf_size.  The two
     * pair lists get 2^18 extra slots on top of the value given: walk waves fill
     * them in blocks of 256 and leave the unused end of their last block empty. */
    int64_t cell_capacity;     /* octree cells */
    int64_t m2l_capacity;      /* well-separated cell pairs of one walk */
    int64_t p2p_capacity;      /* cell pairs treated by direct sums in one walk */
    int64_t queue_capacity;    /* cell pairs visited by one walk (at most 1e8) */
    /* per-target interaction lists, filled by the gravity walk itself; 0 = automatic
     * (2048 M2L partners per cell, 4096 source cells per leaf: enough for clustered
     * disks of 4e6 moonlets at the default thresholds), at most 8192 each.  A target with more entries makes the call
     * fail with NCORP_E_CAPACITY, required = the count that would have fitted. */
    int32_t m2l_per_cell;      /* well-separated partner cells kept per cell */
    int32_t p2p_per_leaf;      /* direct-sum source cells kept per leaf */
    /* collisions in ncorp_step / ncorp_step_batched: NCORP_COLLISIONS_REPORT (0,
     * default) lists every pair found and changes nothing; NCORP_COLLISIONS_RESOLVE
     * (1) also resolves them as hard-sphere impacts (Sect. 5.1-5.2): the impulse
     * J = alpha (dr . dv) dr with alpha = f m1 m2 / ((m1 + m2) (R1 + R2)^2) at the
     * contact time of Eq. (2), f = collision_f in [1, 2] (2: elastic, the default;
     * 1: the normal relative velocity is removed).  A moonlet collides at most once
     * per step: pairs are taken in increasing contact time (ties by i, then j) and
     * a pair is dropped when one of its moonlets has already collided.  Each
     * resolved moonlet moves on its old velocity up to contact and on the new one
     * for the rest of the drift. */
    int32_t collision_mode;
    double collision_f;
    /* central-body extras, added to the central mass in the kicks of ncorp_step
     * (0 disables each; the gravity of ncorp_gravity is unchanged):
     *   J2, R_central: the central body's equatorial bulge, potential
     *     -G M_c R_central^2 J2 (r^2 - 3 z^2) / (2 r^5), its axis along z;
     *   M_sun, a_sun, obliquity: a distant body on a circular orbit of radius a_sun
     *     in the plane tilted by `obliquity` about x, to quadrupolar order, at
     *     longitude lambda = t sqrt(G M_sun / a_sun^3);
     *   t_start: the time of the first ncorp_step call; the context's clock then
     *     advances by n_steps dt per call (on the host, so a captured call replays
     *     the times it was captured with). */
    double J2, R_central;
    double M_sun, a_sun, obliquity;
    double t_start;
    /* gravity method (Sect. 3.4): NCORP_GRAVITY_FALCON (0, default) is the dual
     * walk of Alg. 2 with its cell-cell terms; NCORP_GRAVITY_STANDARD_TREE (1) is
     * the standard tree code of Alg. 1: every moonlet walks the tree from its root
     * on its own, a cell B with fewer than ncb_pre moonlets is summed directly, a
     * cell with |x - s_B| >= r_crit,B contributes its cell-moonlet C^(1) term
     * (orders 0 and 2..p-1 of the multipoles), a cell with fewer than ncb_post
     * moonlets or a leaf is summed directly, and any other cell is opened.  The
     * standard tree computes in FP64 whatever `precision` says, keeps no
     * interaction lists, and leaves collision search to the collision walk.
     * Paper settings: leaf_size 102, ncb_pre 6, ncb_post 16 (Sect. 6). */
    int32_t gravity_method;
    int32_t ncb_pre, ncb_post;
    /* mesh module (Sect. 3.3), used by gravity_method NCORP_GRAVITY_MESH and by
     * collision_method NCORP_COLLISIONS_MESH.  Cubic cells of side gamma, cell
     * (floor(x/gamma), floor(y/gamma), floor(z/gamma)); a moonlet's neighbourhood
     * is its cell and the 26 adjacent ones.  Moonlets in each other's
     * neighbourhood attract each other and are tested for collision; a moonlet
     * with 2R > gamma stays out of the mesh and interacts with every moonlet; for
     * gravity, so do the three most massive moonlets (equal masses: smaller input
     * index first).  Nothing else interacts.  Occupied cells are found through a
     * hash table keyed by the exact cell (2 n_max slots or more, 16 bytes each);
     * cell coordinates must stay within +-(2^20 - 2).
     *   mesh_cells, mesh_min_side: the whole grid spans at least mesh_min_side
     *     with mesh_cells cells per axis, so gamma >= mesh_min_side / mesh_cells;
     *   mesh_neighbours: x, the mean number of neighbours aimed at;
     *   mesh_gamma: the first mesh size; 0 = Eq. (4) with aspect ratio
     *     mesh_aspect and radius mesh_rmax (0 = the largest distance of a moonlet
     *     to the central mass at the first mesh);
     *   every later mesh: gamma = gamma' (x / x')^(1/3) (Eq. 6), x' the mean
     *     number of neighbours of the moonlets of the previous mesh (x' = 0
     *     doubles gamma), and never below mesh_min_side / mesh_cells (1 or more).
     * The mesh size lives in the workspace and restarts from mesh_gamma or Eq. (4)
     * when a new workspace buffer is bound.  Plain (not batched) calls only. */
    int32_t collision_method;
    int32_t mesh_cells;
    double mesh_neighbours, mesh_aspect, mesh_rmax, mesh_min_side, mesh_gamma;
    /* launch shape of the falcON gravity evaluation (results do not depend on the last
     * two; the tile moves the FP32 direct sums' rounding, not their accuracy class):
     *   p2p_tile: source moonlets a direct-sum wave stages in LDS at a time, 128, 256
     *     or 512 (0 = 256);
     *   p2p_targets_max: the most target moonlets one lane of the direct sums holds,
     *     1..4 (0 = 4); each leaf takes the count in 1..max that keeps most lanes busy;
     *   walk_waves: persistent waves of the gravity walk, 256, 512, 1024 or 2048
     *     (0 = 1024); each claims 128 queue items at a time, so this sets how many
     *     items of the walk's queue are in flight. */
    int32_t p2p_tile, p2p_targets_max, walk_waves;
} ncorp_params;

enum { NCORP_COLLISIONS_REPORT = 0, NCORP_COLLISIONS_RESOLVE = 1 };
/* gravity: the falcON walk, the standard tree code, the mesh module, or every pair
 * (Sect. 3.2: the plain sum, O(N^2), on the tree-ordered moonlets of the last build) */
enum {
    NCORP_GRAVITY_FALCON = 0, NCORP_GRAVITY_STANDARD_TREE = 1, NCORP_GRAVITY_MESH = 2,
    NCORP_GRAVITY_BRUTE_FORCE = 3
};
/* collision search: the falcON walk (or the gravity walk's lists of the same tree),
 * the mesh, or the standard tree code's per-moonlet walk (Alg. 1, collision form: a
 * cell whose sphere cannot meet the moonlet's reach R + dt |v| is skipped, other cells
 * are brute-forced below ncb_pre / ncb_post moonlets or at leaves, or opened) */
enum {
    NCORP_COLLISIONS_TREE = 0, NCORP_COLLISIONS_MESH = 1, NCORP_COLLISIONS_STANDARD_TREE = 2,
    NCORP_COLLISIONS_BRUTE_FORCE = 3     /* every pair i < j (Sect. 3.2), O(N^2) */
};

typedef struct ncorp_ctx ncorp_ctx;

/* Defaults from the paper's timing runs (Sect. 4.2): order p with s = 17 and
 * thresholds (64, 8, 64) for p <= 3, s = 52 and (256, 256, 512) above; collision
 * thresholds (12, 0, 16); theta_min = 0.5, mass-dependent theta; G = 1,
 * M_central = 1; FP64.  Returns NCORP_E_INVALID for p outside 0..6. */
int ncorp_params_default(ncorp_params *out, int p);

/* Validates the parameters (p in 0..6, 0 < theta_min < 1, s >= 1, thresholds
 * >= 0, G >= 0) and creates a host-side context.  No device memory is touched. */
int ncorp_create(const ncorp_params *params, ncorp_ctx **out);
void ncorp_destroy(ncorp_ctx *ctx);

/* Bytes of device workspace needed for up to n_max moonlets and a collision
 * pair buffer of pair_capacity entries; -1 on invalid arguments.  The workspace
 * must be 256-byte aligned. */
int64_t ncorp_workspace_bytes(const ncorp_params *params, int64_t n_max,
                              int64_t pair_capacity);

/* Root cube, 63-bit Hilbert keys, stable radix sort by (key, input index) and
 * the flat octree: cells ordered by level, then Hilbert order inside a level,
 * children contiguous (Sect. 3.4.1, Sect. 3.4.6).  x, y, z: n FP64 positions.
 * The tree stays in the workspace for later calls on this context. */
int ncorp_build_tree(ncorp_ctx *ctx, const double *x, const double *y, const double *z,
                     int64_t n, void *workspace, int64_t ws_bytes, void *stream);

/* The mesh of the mesh module (Sect. 3.3, see ncorp_params) at positions x, y, z
 * for moonlets of radii R (n FP64 each): the mesh size for this mesh (Eq. 4 at the
 * first, Eq. 6 after), the cell of every moonlet, the moonlets sorted by the
 * Morton key of their cell, the table of occupied cells.  Needed before ncorp_gravity / ncorp_collide when
 * their method is the mesh (ncorp_step builds it itself).  A cell coordinate
 * beyond +-(2^20 - 2) makes ncorp_get_status return NCORP_E_INVALID; more than 1021
 * moonlets with 2R > gamma, NCORP_E_CAPACITY. */
int ncorp_build_mesh(ncorp_ctx *ctx, const double *x, const double *y, const double *z,
                     const double *R, int64_t n, void *workspace, int64_t ws_bytes,
                     void *stream);

/* Waits for the stream and reports the last mesh: out[0] its mesh size gamma,
 * out[1] the mean number of neighbours x' measured on it (NaN before a gravity or
 * collision pass counted them), out[2] the moonlets in the mesh, out[3] those
 * kept out of it (2R > gamma).  out: 4 doubles, host memory. */
int ncorp_mesh_state(ncorp_ctx *ctx, double *out);

/* Mutual gravitational acceleration of every moonlet: a_i = sum_j G m_j (x_j -
 * x_i)/|x_j - x_i|^3 as approximated by the chosen method -- the falcON walk on
 * the last tree (Eqs. 10-12, 20, 25, 26 and Alg. 2), the standard tree code
 * (Alg. 1), or the mesh module on the last mesh (Sect. 3.3).  m: n masses; ax, ay,
 * az: n outputs, input order.  The central mass is NOT included here. */
int ncorp_gravity(ncorp_ctx *ctx, const double *m, double *ax, double *ay, double *az,
                  void *stream);

/* Collision search (Sect. 3.1) on the last tree (Sect. 3.4.2; every pair i < j
 * whose straight-line trajectories touch at a time 0 <= t <= dt, Eqs. 1-2) or, with
 * collision_method NCORP_COLLISIONS_MESH, on the last mesh (the pairs of
 * neighbours and of moonlets kept out of the mesh that touch, Sect. 3.3).
 * vx, vy, vz, R: n FP64 velocities and radii.  pairs: cap x 2 int64, written in
 * lexicographic order, no duplicates; n_pairs_dev: one int64 (device) receiving the
 * number found (which may exceed cap: then the status is NCORP_E_CAPACITY). */
int ncorp_collide(ncorp_ctx *ctx, const double *vx, const double *vy, const double *vz,
                  const double *R, double dt, int64_t *pairs, int64_t cap,
                  int64_t *n_pairs_dev, void *stream);

/* n_steps of the merged kick-drift-kick leapfrog (Sect. 4.1) around the central
 * mass (App. B.1): the first call builds the tree and gravity at the start state;
 * every step then kicks, searches collisions on (x, v) over dt with the current
 * tree, drifts, rebuilds the tree, recomputes gravity (mutual + central) and
 * kicks.  x..vz are updated in place.  pairs receives (step, i, j) triples,
 * cap x 3 int64, each step's pairs in lexicographic order; n_pairs_dev receives
 * n_steps int64 counts.  With collision_mode NCORP_COLLISIONS_REPORT these are all
 * pairs found and nothing is changed; with NCORP_COLLISIONS_RESOLVE they are the
 * pairs resolved (see ncorp_params). */
int ncorp_step(ncorp_ctx *ctx, double *x, double *y, double *z, double *vx, double *vy,
               double *vz, const double *m, const double *R, int64_t n, double dt,
               int n_steps, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev,
               void *workspace, int64_t ws_bytes, void *stream);

/* ---- batched form: many independent disks in one call ---------------------
 * The moonlets of n_disks independent systems, each around its own central mass
 * at the origin, are concatenated: disk d holds moonlets [off[d], off[d+1]) of
 * every array.  The batched calls compute exactly what the plain call would give
 * for every disk on its own -- one root cube and one tree per disk (a forest whose
 * level 0 holds one root per non-empty disk), a dual walk started from (root,
 * root) of every disk, no term and no pair across disks -- in the same launches
 * for all disks.  Empty disks are allowed.
 *
 * disk_offsets: n_disks + 1 int64 in DEVICE memory, owned by the caller, read by
 * the call's kernels (also on every replay of a captured call); they must be
 * non-decreasing from 0 to n.  This is checked on the device: a violation makes
 * every later kernel of the call do nothing and ncorp_get_status return
 * NCORP_E_INVALID.  1 <= n_disks <= NCORP_MAX_DISKS, checked on the host.
 *
 * Graph capture: these calls (like ncorp_step) only enqueue kernels on `stream`
 * -- no allocation, copy, memset or host synchronisation -- so a call may be
 * captured into a hipGraph and replayed; the walk-queue tags advance on the
 * device, so replays stay valid.  Capture after one eager call on the same
 * workspace (the first walk on a new workspace clears its queue, which would
 * otherwise be captured too), with phase timing off. */
#define NCORP_MAX_DISKS 65536

/* ncorp_build_tree for a batch of disks (Sect. 3.4.1, Sect. 3.4.6, applied per
 * disk).  Later ncorp_gravity / ncorp_collide calls act on the forest. */
int ncorp_build_tree_batched(ncorp_ctx *ctx, const int64_t *disk_offsets, int n_disks,
                             const double *x, const double *y, const double *z, int64_t n,
                             void *workspace, int64_t ws_bytes, void *stream);

/* ncorp_step for a batch of disks (Sect. 4.1, App. B.1, per disk): same arrays,
 * outputs and pair format as ncorp_step; pairs never join two disks. */
int ncorp_step_batched(ncorp_ctx *ctx, const int64_t *disk_offsets, int n_disks, double *x,
                       double *y, double *z, double *vx, double *vy, double *vz,
                       const double *m, const double *R, int64_t n, double dt, int n_steps,
                       int64_t *pairs, int64_t cap, int64_t *n_pairs_dev, void *workspace,
                       int64_t ws_bytes, void *stream);

/* ---- allocation-free form --------------------------------------------------
 * For callers that cannot allocate device memory or bring a workspace: code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc.
 * ncorp_step_noalloc is ncorp_step (same arguments, minus the workspace; same
 * results, pair format and errors) with the workspace taken from a fixed array
 * inside the library, NCORP_STATIC_WORKSPACE_BYTES on every GPU it runs on, set up
 * by the first call on that GPU (the device current at the call) and held until
 * the process ends.  Nothing is allocated or freed by the call.
 *  - Size limit: n must satisfy ncorp_workspace_bytes(params, n, 1) <=
 *    NCORP_STATIC_WORKSPACE_BYTES (with the default capacities up to 18 810 moonlets
 *    at p = 6 and 19 824 at p = 4, leaf size 52, and 7 048 at p = 3, leaf size 17;
 *    a larger leaf size allows more); a larger n returns
 *    NCORP_E_INVALID at once, before anything touches the GPU.  The part of the
 *    array the layout does not use holds the colliding pairs of the step.
 *  - Sharing: all calls on one GPU use that GPU's one array, which keeps the last
 *    call's contents.  Each call starts from cleared device state and uses nothing an
 *    earlier call left, so calls of different contexts may follow each other in
 *    stream order; calls that overlap in time on one GPU (different streams or
 *    threads without ordering between them) race and give undefined results.
 *  - Afterwards ncorp_get_status, ncorp_tree_info and ncorp_export_host on this
 *    context read the array, which is valid only until the next call on that GPU. */
#define NCORP_STATIC_WORKSPACE_BYTES (128LL * 1024 * 1024)
int ncorp_step_noalloc(ncorp_ctx *ctx, double *x, double *y, double *z, double *vx,
                       double *vy, double *vz, const double *m, const double *R, int64_t n,
                       double dt, int n_steps, int64_t *pairs, int64_t cap,
                       int64_t *n_pairs_dev, void *stream);

/* Waits for the context's last stream, then reports the device status word:
 * NCORP_OK, NCORP_E_CAPACITY (required_capacity, if not NULL, receives the size
 * that would have sufficed for the list that overflowed), NCORP_E_INVALID (bad
 * disk offsets of a batched call) or NCORP_E_NONFINITE.
 * The status is cleared by the next ncorp_build_tree / ncorp_step. */
int ncorp_get_status(ncorp_ctx *ctx, int64_t *required_capacity);

/* Last error message of this context (static storage, never NULL). */
const char *ncorp_last_error(const ncorp_ctx *ctx);

/* ---- inspection of the last tree and walks (tests, tuning) ---------------- */
enum {
    NCORP_INFO_N = 0, NCORP_INFO_NCELLS, NCORP_INFO_NLEAVES, NCORP_INFO_MAXLEVEL,
    NCORP_INFO_M2L, NCORP_INFO_P2P, NCORP_INFO_VISITED, NCORP_INFO_COL_CAND,
    NCORP_INFO_COL_TESTS, NCORP_INFO_M2L_DIR, NCORP_INFO_P2P_INTER, NCORP_INFO_M2L_MAXLIST,
    NCORP_INFO_P2P_MAXLIST, NCORP_INFO_NROOTS, NCORP_INFO_LONG_M2L, NCORP_INFO_LONG_P2P,
    NCORP_INFO_WALK_BUSY_MAX, NCORP_INFO_WALK_BUSY_MEAN, NCORP_INFO_P2P_SRC_MAX,
    NCORP_INFO_SORT_PREV, NCORP_INFO_SORT_SPILL,
    NCORP_INFO_COUNT
};
/* Waits for the stream and fills info[NCORP_INFO_COUNT] with sizes of the last
 * tree and walks (cells, leaves, deepest level, M2L and P2P cell pairs of the
 * last gravity walk, visited pairs, collision candidate cell pairs, pair tests
 * performed (moonlets that cannot reach the other cell are culled first),
 * directed M2L interactions, directed moonlet-moonlet interactions of the direct
 * sums with i != j, longest per-target M2L list, longest per-leaf direct-sum list:
 * the sizes m2l_per_cell and p2p_per_leaf must cover; these three are filled
 * only while phase timing is on (ncorp_set_timing), otherwise they read 0), and
 * the number of roots (level-0 cells: 1, or the non-empty disks of a batched
 * call), and the numbers of cells and leaves whose M2L or direct-sum lists were too
 * long for one LDS batch of their consumer (sorted by a pre-pass; the direct sums of
 * such leaves are split over several waves); and, again only while phase timing is on,
 * the load balance of the last gravity evaluation: the largest and the mean number of
 * shader clock cycles (clock64) the gravity walk's persistent waves were busy, and the
 * most source moonlets of one leaf's direct sums (the mean is p2p_inter / n).  The
 * last two describe the sort of the last plain tree build (Sect. 3.4.6): 1 if its
 * buckets came from the order of the build before it (0: from a sample of the keys),
 * and the number of buckets too large for one LDS batch, sorted by merging. */
int ncorp_tree_info(ncorp_ctx *ctx, int64_t *info);

enum {
    NCORP_EXPORT_KEYS = 0,     /* n uint64: sorted Hilbert keys */
    NCORP_EXPORT_PERM,         /* n int32: tree position -> input index */
    NCORP_EXPORT_CELLS,        /* ncells x 8 int32: level, first, count,
                                  child_first (-1 for leaves), nchild, parent,
                                  prefix low 32 bits, prefix high 32 bits */
    NCORP_EXPORT_GCELLS,       /* ncells x 8 double: sx, sy, sz, mass, r_max,
                                  r_crit, theta, 0 (gravity climb) */
    NCORP_EXPORT_CCELLS,       /* ncells x 4 double: sbar x, y, z, r_crit
                                  (collision climb); r_max follows as a second
                                  block of ncells doubles */
    NCORP_EXPORT_MULTIPOLES,   /* ncells x nm double: M^(n)_a / a! for n = 0, 2..p-1,
                                  components ordered by order, then (ax, ay, az)
                                  with ax descending, then ay descending */
    NCORP_EXPORT_LOCAL,        /* ncells x nc double: C^(m)_a after the walk, m = 1..p,
                                  same component order (before the descent) */
    NCORP_EXPORT_M2L,          /* nm2l x 2 int32 cell pairs of the gravity walk */
    NCORP_EXPORT_P2P,          /* np2p x 2 int32 cell pairs of the gravity walk */
    NCORP_EXPORT_COL_CAND,     /* ncand x 2 int32 cell pairs of the collision walk */
    NCORP_EXPORT_COUNT
};
/* Copies an internal array to host memory `dst` of `bytes` bytes (waits for the
 * stream).  Returns the number of bytes the full array needs (copying at most
 * `bytes`), or a negative ncorp_status. */
int64_t ncorp_export_host(ncorp_ctx *ctx, int what, void *dst, int64_t bytes);

/* ---- phase timing (benchmarks) -------------------------------------------- */
enum {
    NCORP_PHASE_KEYS = 0, NCORP_PHASE_SORT, NCORP_PHASE_TREE, NCORP_PHASE_GCLIMB,
    NCORP_PHASE_GWALK, NCORP_PHASE_M2L, NCORP_PHASE_DESCENT,
    NCORP_PHASE_P2P, NCORP_PHASE_L2P, NCORP_PHASE_COLLIDE, NCORP_PHASE_INTEGRATE,
    NCORP_PHASE_COUNT
};
/* enable != 0: every later call records a HIP event pair on its stream around each
 * phase (the P2P phase is exactly one kernel launch).  Costs a few microseconds per
 * phase; off by default. */
int ncorp_set_timing(ncorp_ctx *ctx, int enable);
/* Waits for the recorded events and adds, per phase, the elapsed milliseconds to
 * ms[NCORP_PHASE_COUNT] and the number of recorded launches to count[...]; then
 * forgets the records.  Either pointer may be NULL. */
int ncorp_phase_times(ncorp_ctx *ctx, double *ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* NCORP_H */

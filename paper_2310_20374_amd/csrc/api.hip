// Host side of libncorp: argument checks, workspace layout and the order in which
// the kernels of one call are enqueued.  Nothing here allocates device memory and
// nothing waits for the GPU except the status / inspection calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "ncorp_internal.h"

using namespace ncorp;

struct PhaseRec {
    int phase;
    hipEvent_t a, b;
};

struct ncorp_ctx {
    ncorp_params prm;
    Workspace ws;
    bool have_tree = false;
    int64_t n = 0;
    double clock = 0.0;                 // time of the next ncorp_step call
    bool grav_lists = false;            // the gravity walk ran on the current tree
    bool have_mesh = false;             // a mesh was built (mesh module)
    bool mesh_init = false;             // the workspace's mesh state has been set up
    bool mesh_counted = false;          // neighbours counted on the current mesh
    hipStream_t last = nullptr;
    char err[256];
    // phase timing
    bool timing = false;
    std::vector<hipEvent_t> pool;
    std::vector<PhaseRec> recs;
    ~ncorp_ctx() {
        for (auto &r : recs) { pool.push_back(r.a); pool.push_back(r.b); }
        for (auto e : pool) hipEventDestroy(e);
    }
};

// Records an event pair around one phase when timing is on.
struct PhaseTimer {
    ncorp_ctx *c;
    hipStream_t s;
    PhaseRec rec{};
    bool on;
    PhaseTimer(ncorp_ctx *c_, int phase, hipStream_t s_) : c(c_), s(s_), on(c_->timing) {
        if (!on) return;
        rec.phase = phase;
        rec.a = take();
        rec.b = take();
        if (!rec.a || !rec.b) { on = false; return; }
        hipEventRecord(rec.a, s);
    }
    hipEvent_t take() {
        if (!c->pool.empty()) { hipEvent_t e = c->pool.back(); c->pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    ~PhaseTimer() {
        if (!on) return;
        hipEventRecord(rec.b, s);
        c->recs.push_back(rec);
    }
};

static int fail(ncorp_ctx *c, int code, const char *msg) {
    if (c) std::snprintf(c->err, sizeof(c->err), "%s", msg);
    return code;
}

static int hip_fail(ncorp_ctx *c, hipError_t e, const char *where) {
    if (c)
        std::snprintf(c->err, sizeof(c->err), "%s: %s", where, hipGetErrorString(e));
    return NCORP_E_HIP;
}

#define HIPCHK(ctx, expr)                                      \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

static bool params_ok(const ncorp_params *p, char *why, size_t len) {
    if (!p) { std::snprintf(why, len, "params is NULL"); return false; }
    if (p->p < 0 || p->p > kMaxP) { std::snprintf(why, len, "p must be in 0..6"); return false; }
    if (!(p->theta_min > 0.0 && p->theta_min < 1.0)) {
        std::snprintf(why, len, "theta_min must be in (0, 1)"); return false;
    }
    if (p->theta_mode != 0 && p->theta_mode != 1) {
        std::snprintf(why, len, "theta_mode must be 0 or 1"); return false;
    }
    if (p->leaf_size < 1 || p->leaf_size > 1024) {
        std::snprintf(why, len, "leaf_size must be in 1..1024"); return false;
    }
    if (p->ncs < 0 || p->ncc_pre < 0 || p->ncc_post < 0 || p->ncs_col < 0 ||
        p->ncc_pre_col < 0 || p->ncc_post_col < 0) {
        std::snprintf(why, len, "walk thresholds must be >= 0"); return false;
    }
    if (!(p->G >= 0.0) || !(p->M_central >= 0.0)) {
        std::snprintf(why, len, "G and M_central must be >= 0"); return false;
    }
    if (p->precision != NCORP_FP64 && p->precision != NCORP_FP32_BULK) {
        std::snprintf(why, len, "unknown precision"); return false;
    }
    if (!(p->root_half_width >= 0.0)) {
        std::snprintf(why, len, "root_half_width must be >= 0"); return false;
    }
    if (p->root_half_width > 0.0) {
        int e;
        double f = std::frexp(p->root_half_width, &e);
        if (f != 0.5) { std::snprintf(why, len, "root_half_width must be a power of two"); return false; }
    }
    if (p->cell_capacity < 0 || p->m2l_capacity < 0 || p->p2p_capacity < 0 ||
        p->queue_capacity < 0) {
        std::snprintf(why, len, "capacities must be >= 0"); return false;
    }
    if (p->queue_capacity > kMaxQueue) {
        std::snprintf(why, len, "queue_capacity must be at most %lld", (long long)kMaxQueue);
        return false;
    }
    if (p->m2l_per_cell < 0 || p->m2l_per_cell > kMaxPerTarget || p->p2p_per_leaf < 0 ||
        p->p2p_per_leaf > kMaxPerTarget) {
        std::snprintf(why, len, "m2l_per_cell and p2p_per_leaf must be in 0..%d", kMaxPerTarget);
        return false;
    }
    if (p->collision_mode != NCORP_COLLISIONS_REPORT &&
        p->collision_mode != NCORP_COLLISIONS_RESOLVE) {
        std::snprintf(why, len, "collision_mode must be 0 or 1"); return false;
    }
    if (!(p->collision_f >= 1.0 && p->collision_f <= 2.0)) {
        std::snprintf(why, len, "collision_f must be in [1, 2]"); return false;
    }
    if (!std::isfinite(p->J2) || (p->J2 != 0.0 && !(p->R_central > 0.0))) {
        std::snprintf(why, len, "J2 needs a finite value and R_central > 0"); return false;
    }
    if (!(p->M_sun >= 0.0) || (p->M_sun > 0.0 && !(p->a_sun > 0.0)) ||
        !std::isfinite(p->obliquity) || !std::isfinite(p->t_start)) {
        std::snprintf(why, len, "M_sun >= 0 (then a_sun > 0), finite obliquity and t_start");
        return false;
    }
    if (p->gravity_method != NCORP_GRAVITY_FALCON &&
        p->gravity_method != NCORP_GRAVITY_STANDARD_TREE &&
        p->gravity_method != NCORP_GRAVITY_MESH &&
        p->gravity_method != NCORP_GRAVITY_BRUTE_FORCE) {
        std::snprintf(why, len, "gravity_method must be 0..3"); return false;
    }
    if (p->ncb_pre < 0 || p->ncb_post < 0) {
        std::snprintf(why, len, "ncb_pre and ncb_post must be >= 0"); return false;
    }
    if (p->collision_method != NCORP_COLLISIONS_TREE &&
        p->collision_method != NCORP_COLLISIONS_MESH &&
        p->collision_method != NCORP_COLLISIONS_STANDARD_TREE &&
        p->collision_method != NCORP_COLLISIONS_BRUTE_FORCE) {
        std::snprintf(why, len, "collision_method must be 0..3"); return false;
    }
    if (p->mesh_cells < 1) {
        std::snprintf(why, len, "mesh_cells must be >= 1"); return false;
    }
    if (!(p->mesh_neighbours > 0.0 && std::isfinite(p->mesh_neighbours)) ||
        !(p->mesh_aspect >= 0.0 && std::isfinite(p->mesh_aspect)) ||
        !(p->mesh_rmax >= 0.0 && std::isfinite(p->mesh_rmax)) ||
        !(p->mesh_min_side >= 0.0 && std::isfinite(p->mesh_min_side)) ||
        !(p->mesh_gamma >= 0.0 && std::isfinite(p->mesh_gamma))) {
        std::snprintf(why, len, "mesh_neighbours > 0; mesh_aspect, mesh_rmax, mesh_min_side, "
                                "mesh_gamma finite and >= 0");
        return false;
    }
    if (p->mesh_gamma == 0.0 && p->mesh_aspect == 0.0 && p->mesh_min_side == 0.0) {
        std::snprintf(why, len, "Eq. (4) needs mesh_aspect > 0 (or give mesh_gamma)");
        return false;
    }
    if (p->p2p_tile != 0 && p->p2p_tile != 128 && p->p2p_tile != 256 && p->p2p_tile != 512) {
        std::snprintf(why, len, "p2p_tile must be 0, 128, 256 or 512"); return false;
    }
    if (p->p2p_targets_max < 0 || p->p2p_targets_max > 4) {
        std::snprintf(why, len, "p2p_targets_max must be in 0..4"); return false;
    }
    if (p->walk_waves != 0 && p->walk_waves != 256 && p->walk_waves != 512 &&
        p->walk_waves != 1024 && p->walk_waves != kWalkWavesMax) {
        std::snprintf(why, len, "walk_waves must be 0, 256, 512, 1024 or 2048"); return false;
    }
    return true;
}

extern "C" int ncorp_params_default(ncorp_params *o, int p) {
    if (!o || p < 0 || p > kMaxP) return NCORP_E_INVALID;
    std::memset(o, 0, sizeof(*o));
    o->G = 1.0;
    o->M_central = 1.0;
    o->p = p;
    o->theta_min = 0.5;
    o->theta_mode = 0;
    if (p <= 3) { o->leaf_size = 17; o->ncs = 64; o->ncc_pre = 8; o->ncc_post = 64; }
    else { o->leaf_size = 52; o->ncs = 256; o->ncc_pre = 256; o->ncc_post = 512; }
    o->ncs_col = 12; o->ncc_pre_col = 0; o->ncc_post_col = 16;
    o->precision = NCORP_FP64;
    o->root_half_width = 0.0;
    o->collision_mode = NCORP_COLLISIONS_REPORT;
    o->collision_f = 2.0;
    o->J2 = 0.0;
    o->R_central = 1.0;
    o->M_sun = 0.0;
    o->a_sun = 0.0;
    o->obliquity = 0.0;
    o->t_start = 0.0;
    o->gravity_method = NCORP_GRAVITY_FALCON;
    o->ncb_pre = 6;
    o->ncb_post = 16;
    o->collision_method = NCORP_COLLISIONS_TREE;
    o->mesh_cells = 256;
    o->mesh_neighbours = 8.0;
    o->mesh_aspect = 0.05;
    o->mesh_rmax = 0.0;
    o->mesh_min_side = 0.0;
    o->mesh_gamma = 0.0;
    o->p2p_tile = 0;
    o->p2p_targets_max = 0;
    o->walk_waves = 0;
    return NCORP_OK;
}

extern "C" int ncorp_create(const ncorp_params *params, ncorp_ctx **out) {
    char why[128];
    if (!out) return NCORP_E_INVALID;
    *out = nullptr;
    if (!params_ok(params, why, sizeof(why))) return NCORP_E_INVALID;
    ncorp_ctx *c = new ncorp_ctx();
    c->prm = *params;
    c->clock = params->t_start;
    c->err[0] = 0;
    *out = c;
    return NCORP_OK;
}

extern "C" void ncorp_destroy(ncorp_ctx *c) { delete c; }

extern "C" const char *ncorp_last_error(const ncorp_ctx *c) {
    return c ? c->err : "no context";
}

// ------------------------------------------------------------------ layout
namespace ncorp {

static int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

int64_t layout_workspace(Workspace &ws, const ncorp_params &prm, int64_t n_max, int64_t pair_cap) {
    const int64_t n = n_max < 1 ? 1 : n_max;
    const int s = prm.leaf_size;
    int64_t cell_cap = prm.cell_capacity > 0 ? prm.cell_capacity : 8 * n / s + 1024;
    if (cell_cap > (1 << 24) - 2) cell_cap = (1 << 24) - 2;
    // plain pair lists: entries plus at most one partly used chunk per walk wave (the
    // gravity walk's waves, or the collision walk's if it runs more)
    const int collide_waves = kWalkGridCollide * (kWalkBlock / kWave);
    const int64_t slack =
        (int64_t)(walk_waves(prm) > collide_waves ? walk_waves(prm) : collide_waves) * kListChunk;
    int64_t m2l_cap = (prm.m2l_capacity > 0 ? prm.m2l_capacity : 64 * cell_cap + 4096) + slack;
    int64_t p2p_cap = (prm.p2p_capacity > 0 ? prm.p2p_capacity : 32 * cell_cap + 4096) + slack;
    int64_t q_cap = prm.queue_capacity > 0 ? prm.queue_capacity
                                           : m2l_cap + p2p_cap + 16 * cell_cap + 65536;
    if (q_cap > kMaxQueue) q_cap = kMaxQueue;
    ws.n_max = n;
    ws.cell_cap = cell_cap;
    ws.m2l_cap = m2l_cap;
    ws.p2p_cap = p2p_cap;
    ws.queue_cap = q_cap;
    ws.leaf_cap = cell_cap < n ? cell_cap : n;
    ws.m2l_stride = prm.m2l_per_cell > 0 ? prm.m2l_per_cell : kDefaultM2LPerCell;
    ws.p2p_stride = prm.p2p_per_leaf > 0 ? prm.p2p_per_leaf : kDefaultP2PPerLeaf;
    ws.pair_cap = pair_cap < 1 ? 1 : pair_cap;
    ws.p = prm.p;
    ws.nm = n_mult(prm.p);
    ws.nl = n_local(prm.p);
    const int64_t nb = (n + 1023) / 1024;
    const int64_t ntiles = (n + kSortTileItems - 1) / kSortTileItems;
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        int64_t o = off;
        off += align256(bytes < 8 ? 8 : bytes);
        return ws.base ? (void *)(ws.base + o) : nullptr;
    };
    ws.st = (DevState *)take(sizeof(DevState));
    ws.wq = (WalkQueue *)take(sizeof(WalkQueue));
    ws.keys = (uint64_t *)take(8 * n);
    ws.keys_alt = (uint64_t *)take(8 * n);
    ws.idx = (uint32_t *)take(4 * n);
    ws.idx_alt = (uint32_t *)take(4 * n);
    ws.code = (uint32_t *)take(4 * n);
    ws.pack4 = (double4 *)take(32 * n);
    ws.xs = (double *)take(8 * n);
    ws.ys = (double *)take(8 * n);
    ws.zs = (double *)take(8 * n);
    ws.mus = (double *)take(8 * n);
    ws.vxs = (double *)take(8 * n);
    ws.vys = (double *)take(8 * n);
    ws.vzs = (double *)take(8 * n);
    ws.rads = (double *)take(8 * n);
    ws.pcol = (double4 *)take(32 * n);
    ws.cbox = (double4 *)take(2 * 32 * cell_cap);
    ws.vcol = (double4 *)take(32 * n);
    ws.acc = (double *)take(3 * 8 * n);
    ws.acc_s = (double *)take(3 * 8 * n);
    ws.ent_start = (int32_t *)take(4 * n);
    ws.ent_code = (uint32_t *)take(4 * n);
    ws.ent_cell = (int32_t *)take(4 * n);
    ws.c_level = (int32_t *)take(4 * cell_cap);
    ws.c_first = (int32_t *)take(4 * cell_cap);
    ws.c_count = (int32_t *)take(4 * cell_cap);
    ws.c_child = (int32_t *)take(4 * cell_cap);
    ws.c_nchild = (int32_t *)take(4 * cell_cap);
    ws.c_parent = (int32_t *)take(4 * cell_cap);
    ws.c_entry = (int32_t *)take(4 * cell_cap);
    ws.c_nent = (int32_t *)take(4 * cell_cap);
    ws.c_prefix = (uint64_t *)take(8 * cell_cap);
    ws.c_arrive = (int32_t *)take(4 * cell_cap);
    ws.climb_next = (int32_t *)take(4 * kXcds * 32);
    ws.gcell = (double4 *)take(32 * cell_cap);
    ws.c_mass = (double *)take(8 * cell_cap);
    ws.c_rmax = (double *)take(8 * cell_cap);
    ws.c_theta = (double *)take(8 * cell_cap);
    ws.mult = (double *)take(8 * cell_cap * (ws.nm > 0 ? ws.nm : 1));
    ws.mult32 = (float *)take(4 * cell_cap * (ws.nm > 0 ? ws.nm : 1));
    ws.local = (double *)take(8 * cell_cap * (ws.nl > 0 ? ws.nl : 1));
    ws.cleaf = (double *)take(8 * ws.leaf_cap * (ws.nl > 0 ? ws.nl : 1));
    ws.ccell = (double4 *)take(32 * cell_cap);
    ws.c_crmax = (double *)take(8 * cell_cap);
    ws.wg = (WCell *)take(sizeof(WCell) * cell_cap);
    ws.wc = (WCell *)take(sizeof(WCell) * cell_cap);
    ws.queue = (uint64_t *)take(8 * q_cap);
    ws.m2l = (int2 *)take(8 * m2l_cap);
    ws.p2p = (int2 *)take(8 * p2p_cap);
    ws.cand = (int2 *)take(8 * p2p_cap);
    if (ws.p > 0) {
        ws.m2l_cnt = (int32_t *)take(4 * cell_cap);
        ws.m2l_seg = (int32_t *)take(4 * cell_cap * (int64_t)ws.m2l_stride);
        ws.p2p_cnt = (int32_t *)take(4 * ws.leaf_cap);
        ws.p2p_seg = (int32_t *)take(4 * ws.leaf_cap * (int64_t)ws.p2p_stride);
        ws.long_m2l = (int32_t *)take(4 * cell_cap);
        ws.long_p2p = (int32_t *)take(4 * ws.leaf_cap);
        ws.p2p_part = (double *)take(8 * (int64_t)kLongSlots * 3 * n);
    }
    const int64_t cnt = nb * (kMaxDepth + 1) + 1;
    ws.cnt_a = (int32_t *)take(4 * cnt);
    ws.scan_part = (int32_t *)take(4 * (nb + 4096));
    ws.hist = (uint32_t *)take(4 * 256 * (ntiles + 1));
    {
        int64_t nbk = (n + kBucketMean - 1) / kBucketMean;
        if (nbk > kMaxBuckets) nbk = kMaxBuckets;
        const int64_t nbt = (n + kBucketTile - 1) / kBucketTile;
        ws.bs_split = (SplitKey *)take(sizeof(SplitKey) * nbk);
        ws.bs_prev = (SplitKey *)take(sizeof(SplitKey) * nbk);
        const int64_t nsub = (n + kSubStride - 1) / kSubStride;
        ws.bs_sub[0] = (SplitKey *)take(sizeof(SplitKey) * nsub);
        ws.bs_sub[1] = (SplitKey *)take(sizeof(SplitKey) * nsub);
        ws.bs_cm = (uint32_t *)take(4 * nbk * nbt);
        ws.bs_total = (uint32_t *)take(4 * nbk);
        ws.bs_off = (uint32_t *)take(4 * (nbk + 1));
        ws.bs_done = (uint32_t *)take(4 * nbk);
    }
    ws.seg = (uint16_t *)take(2 * n);
    ws.disk_max = (unsigned long long *)take(8 * (int64_t)kMaxDisks);
    ws.disk_L = (double *)take(8 * (int64_t)kMaxDisks);
    ws.disk_root = (int32_t *)take(4 * (int64_t)kMaxDisks);
    ws.pairs_tmp = (int64_t *)take(8 * ws.pair_cap);
    ws.pairs_alt = (int64_t *)take(8 * ws.pair_cap);
    ws.pair_dt = (double *)take(8 * ws.pair_cap);
    ws.pair_flag = (int32_t *)take(4 * ws.pair_cap);
    ws.mbest = (int32_t *)take(4 * n);
    ws.mmatch = (int32_t *)take(4 * n);
    ws.cand_blk = (int32_t *)take(4 * 8192);
    // per-block partials: the box pass's 16384 and the pair tests' kCollideGrid blocks,
    // 2 per mesh block plus 1024, or one per standard-tree wave, whichever needs most
    static_assert(kCollideGrid <= 2 * 16384 + 1024 + 128, "pair-test partials must fit");
    ws.count_part_n = n / 64 + 2 * 16384 + 1024 + 128;
    ws.count_part = (unsigned long long *)take(8 * ws.count_part_n);
    if (prm.gravity_method == NCORP_GRAVITY_MESH ||
        prm.collision_method == NCORP_COLLISIONS_MESH) {
        ws.mtab_n = 1024;
        while (ws.mtab_n < 2 * n) ws.mtab_n *= 2;
        ws.mesh = (MeshState *)take(sizeof(MeshState));
        ws.mtab = (MeshSlot *)take(sizeof(MeshSlot) * ws.mtab_n);
        ws.mgrid_n = 32 * n > (1 << 20) ? 32 * n : (1 << 20);
        ws.mgrid = (int2 *)take(8 * ws.mgrid_n);
        ws.mkeys = (uint64_t *)take(8 * n);
        ws.mkeys_alt = (uint64_t *)take(8 * n);
        ws.midx = (uint32_t *)take(4 * n);
        ws.midx_alt = (uint32_t *)take(4 * n);
        ws.mpos = (double4 *)take(32 * n);
        ws.mcell = (int4 *)take(16 * n);
        ws.mvel = (double4 *)take(32 * n);
        ws.mbig = (int32_t *)take(4 * (int64_t)kMaxMeshBig);
        ws.mmass = (double *)take(8 * n);
        ws.mtop_part = take(16 * 3 * 256);
        ws.mbig_part = (double *)take(8 * 3 * 64 * (int64_t)kMaxMeshBig);
    }
    ws.bytes = off;
    return off;
}

}  // namespace ncorp

extern "C" int64_t ncorp_workspace_bytes(const ncorp_params *params, int64_t n_max,
                                         int64_t pair_capacity) {
    char why[128];
    if (!params_ok(params, why, sizeof(why)) || n_max < 1 || n_max > INT32_MAX - 1 ||
        pair_capacity < 0)
        return -1;
    Workspace w;
    return layout_workspace(w, *params, n_max, pair_capacity);
}

// Fit the layout for n moonlets into the caller's buffer: whatever is left after
// the fixed part becomes the colliding-pair buffer.
static int setup_workspace(ncorp_ctx *c, int64_t n, void *workspace, int64_t ws_bytes) {
    if (!workspace) return fail(c, NCORP_E_INVALID, "workspace is NULL");
    if (((uintptr_t)workspace & 255u) != 0)
        return fail(c, NCORP_E_INVALID, "workspace must be 256-byte aligned");
    Workspace probe;
    const int64_t fixed = layout_workspace(probe, c->prm, n, 1);
    if (ws_bytes < fixed) {
        std::snprintf(c->err, sizeof(c->err), "workspace too small: %lld bytes needed for n=%lld",
                      (long long)fixed, (long long)n);
        return NCORP_E_INVALID;
    }
    // whatever is left beyond the fixed part holds colliding pairs (2 x 8 bytes each)
    int64_t pc = 1 + (ws_bytes - fixed) / kPairBytes;
    if (pc > INT32_MAX) pc = INT32_MAX;           // pair indices are 32-bit
    while (pc > 1 && layout_workspace(probe, c->prm, n, pc) > ws_bytes) pc -= pc > 64 ? 64 : 1;
    Workspace ws;
    ws.base = (char *)workspace;
    layout_workspace(ws, c->prm, n, pc);
    // the walk queue keeps tags from earlier walks; a new buffer or layout holds
    // unknown bytes, so the next walk clears it
    ws.clear_queue = !(c->ws.base == ws.base && c->ws.queue == ws.queue &&
                       c->ws.queue_cap == ws.queue_cap) || c->ws.clear_queue;
    // the bucket sort's boundaries from the last build are usable only where it wrote them
    ws.sort_prev = c->ws.base == ws.base && c->ws.bs_prev == ws.bs_prev && c->ws.sort_prev;
    // so are the cleared climb counters
    ws.arrive_clean = c->ws.base == ws.base && c->ws.c_arrive == ws.c_arrive &&
                      c->ws.climb_next == ws.climb_next && c->ws.arrive_clean;
    // so does the mesh state
    if (ws.mesh) {
        // the O(N) grid clear reads the last dense build's keys and grid: every mesh
        // buffer must be where it was
        const bool same = c->ws.base == ws.base && c->ws.mesh == ws.mesh &&
                          c->ws.mtab == ws.mtab && c->ws.mtab_n == ws.mtab_n &&
                          c->ws.mgrid == ws.mgrid && c->ws.mgrid_n == ws.mgrid_n &&
                          c->ws.mkeys == ws.mkeys && c->ws.midx == ws.midx && c->mesh_init;
        ws.clear_mesh = !same || c->ws.clear_mesh;
        if (!same) { c->mesh_init = false; c->have_mesh = false; }
    }
    c->ws = ws;
    return NCORP_OK;
}

// disk_off: device offsets of a batched call (n_disks + 1 of them), or nullptr;
// m: the masses, when the caller has them (the step): G m then comes into tree order
// with the positions (ws.mus), and the step's gravity evaluation on this tree skips
// its own gather
static int build_tree_impl(ncorp_ctx *c, const double *x, const double *y, const double *z,
                           int64_t n, hipStream_t s, bool fresh, const int64_t *disk_off,
                           int n_disks, const double *m = nullptr, bool max_ready = false) {
    Workspace &ws = c->ws;
    ws.ndisks = disk_off ? n_disks : 1;
    {
        PhaseTimer t(c, NCORP_PHASE_KEYS, s);
        // a rebuild needs only max_abs cleared, which the last build's cell-range pass
        // did (max_ready: a step's drift has since formed it)
        if (fresh) HIPCHK(c, launch_reset_state(ws, s));
        HIPCHK(c, launch_keys(ws, x, y, z, n, c->prm.root_half_width,
                              disk_off ? disk_off : nullptr, m, c->prm.G, s, max_ready));
    }
    {
        PhaseTimer t(c, NCORP_PHASE_SORT, s);
        if (bucket_sort_applies(ws, n)) {
            HIPCHK(c, launch_bucket_sort(ws, n, s));
            ws.sort_prev = true;
        } else {
            HIPCHK(c, launch_sort(ws, n, s));
        }
    }
    {
        PhaseTimer t(c, NCORP_PHASE_TREE, s);
        HIPCHK(c, launch_gather_pos(ws, n, m != nullptr, s));
        HIPCHK(c, launch_build_tree(ws, n, c->prm.leaf_size, s));
        ws.arrive_clean = true;       // its cell-range pass cleared the climbs' counters
    }
    c->have_tree = true;
    c->grav_lists = false;
    c->n = n;
    c->last = s;
    return NCORP_OK;
}

extern "C" int ncorp_build_tree(ncorp_ctx *c, const double *x, const double *y, const double *z,
                                int64_t n, void *workspace, int64_t ws_bytes, void *stream) {
    if (!c) return NCORP_E_INVALID;
    if (!x || !y || !z) return fail(c, NCORP_E_INVALID, "position pointer is NULL");
    if (n < 1 || n > INT32_MAX - 1) return fail(c, NCORP_E_INVALID, "n must be in 1..2^31-2");
    int r = setup_workspace(c, n, workspace, ws_bytes);
    if (r != NCORP_OK) return r;
    return build_tree_impl(c, x, y, z, n, (hipStream_t)stream, true, nullptr, 1);
}

static bool mesh_gravity(const ncorp_params &p) {
    return p.gravity_method == NCORP_GRAVITY_MESH;
}
static bool mesh_collisions(const ncorp_params &p) {
    return p.collision_method == NCORP_COLLISIONS_MESH;
}

// fresh: also reset the device state (no tree build precedes this one)
static int build_mesh_impl(ncorp_ctx *c, const double *x, const double *y, const double *z,
                           const double *R, int64_t n, hipStream_t s, bool fresh) {
    Workspace &ws = c->ws;
    PhaseTimer t(c, NCORP_PHASE_TREE, s);
    if (fresh) HIPCHK(c, launch_reset_state(ws, s));
    HIPCHK(c, launch_mesh_build(ws, x, y, z, R, n, c->prm, !c->mesh_init, s));
    ws.clear_mesh = false;
    c->mesh_init = true;
    c->have_mesh = true;
    c->mesh_counted = false;
    c->n = n;
    c->last = s;
    return NCORP_OK;
}

extern "C" int ncorp_build_mesh(ncorp_ctx *c, const double *x, const double *y, const double *z,
                                const double *R, int64_t n, void *workspace, int64_t ws_bytes,
                                void *stream) {
    if (!c) return NCORP_E_INVALID;
    if (!x || !y || !z || !R) return fail(c, NCORP_E_INVALID, "array pointer is NULL");
    if (n < 1 || n > INT32_MAX - 1) return fail(c, NCORP_E_INVALID, "n must be in 1..2^31-2");
    if (!mesh_gravity(c->prm) && !mesh_collisions(c->prm))
        return fail(c, NCORP_E_INVALID, "no method of this context uses the mesh");
    int r = setup_workspace(c, n, workspace, ws_bytes);
    if (r != NCORP_OK) return r;
    const bool tree_too = !mesh_gravity(c->prm) || !mesh_collisions(c->prm);
    return build_mesh_impl(c, x, y, z, R, n, (hipStream_t)stream, !tree_too);
}

extern "C" int ncorp_mesh_state(ncorp_ctx *c, double *out) {
    if (!c || !out) return NCORP_E_INVALID;
    if (!c->have_mesh || !c->ws.mesh) return fail(c, NCORP_E_INVALID, "no mesh built yet");
    HIPCHK(c, hipStreamSynchronize(c->last));
    MeshState h;
    HIPCHK(c, hipMemcpy(&h, c->ws.mesh, sizeof(MeshState), hipMemcpyDeviceToHost));
    out[0] = h.gamma;
    out[1] = h.measured ? (h.n_in > 0 ? (double)h.nbr_sum / (double)h.n_in : 0.0) : NAN;
    out[2] = (double)h.n_in;
    out[3] = (double)(c->n - h.n_in);
    return NCORP_OK;
}

static int check_disks(ncorp_ctx *c, const int64_t *disk_offsets, int n_disks) {
    if (!disk_offsets) return fail(c, NCORP_E_INVALID, "disk_offsets is NULL");
    if (n_disks < 1 || n_disks > NCORP_MAX_DISKS)
        return fail(c, NCORP_E_INVALID, "n_disks must be in 1..NCORP_MAX_DISKS");
    return NCORP_OK;
}

extern "C" int ncorp_build_tree_batched(ncorp_ctx *c, const int64_t *disk_offsets, int n_disks,
                                        const double *x, const double *y, const double *z,
                                        int64_t n, void *workspace, int64_t ws_bytes,
                                        void *stream) {
    if (!c) return NCORP_E_INVALID;
    int r = check_disks(c, disk_offsets, n_disks);
    if (r != NCORP_OK) return r;
    if (!x || !y || !z) return fail(c, NCORP_E_INVALID, "position pointer is NULL");
    if (n < 1 || n > INT32_MAX - 1) return fail(c, NCORP_E_INVALID, "n must be in 1..2^31-2");
    r = setup_workspace(c, n, workspace, ws_bytes);
    if (r != NCORP_OK) return r;
    return build_tree_impl(c, x, y, z, n, (hipStream_t)stream, true, disk_offsets, n_disks);
}

// mus_packed: the build of the current tree already put G m in ws.mus (the step)
// Does a gravity evaluation end in the falcON L2P pass (which can write packed records)?
static bool gravity_by_l2p(const ncorp_params &p) {
    return p.p > 0 && p.gravity_method == NCORP_GRAVITY_FALCON;
}

// acc4 (falcON evaluations, gravity_by_l2p): the accelerations as (ax, ay, az, 0)
// records in input order instead of the three arrays
static int gravity_impl(ncorp_ctx *c, const double *m, double *ax, double *ay, double *az,
                        hipStream_t s, bool mus_packed = false, double4 *acc4 = nullptr) {
    if (!gravity_by_l2p(c->prm)) acc4 = nullptr;
    Workspace &ws = c->ws;
    const int64_t n = c->n;
    if (c->prm.p == 0) {
        HIPCHK(c, launch_fill_i64((int64_t *)ax, 0, n, s));
        HIPCHK(c, launch_fill_i64((int64_t *)ay, 0, n, s));
        HIPCHK(c, launch_fill_i64((int64_t *)az, 0, n, s));
        return NCORP_OK;
    }
    if (c->prm.gravity_method == NCORP_GRAVITY_BRUTE_FORCE) {
        if (ws.ndisks > 1)
            return fail(c, NCORP_E_UNSUPPORTED, "brute-force gravity takes plain calls only");
        PhaseTimer t(c, NCORP_PHASE_P2P, s);
        HIPCHK(c, launch_gather_scaled(ws, m, c->prm.G, ws.mus, n, s));
        HIPCHK(c, launch_brute_gravity(ws, n, ax, ay, az, s));
        c->grav_lists = false;
        c->last = s;
        return NCORP_OK;
    }
    if (mesh_gravity(c->prm)) {
        PhaseTimer t(c, NCORP_PHASE_GWALK, s);
        HIPCHK(c, launch_mesh_gravity(ws, m, c->prm.G, n, !c->mesh_counted, ax, ay, az, s));
        c->mesh_counted = true;
        c->last = s;
        return NCORP_OK;
    }
    {
        PhaseTimer t(c, NCORP_PHASE_GCLIMB, s);
        if (!mus_packed) HIPCHK(c, launch_gather_scaled(ws, m, c->prm.G, ws.mus, n, s));
        const bool reset = !ws.arrive_clean;
        ws.arrive_clean = false;
        // falcON: the walk's init pass forms the critical radii
        HIPCHK(c, launch_gravity_climb(ws, n, c->prm, s, reset,
                                       c->prm.gravity_method == NCORP_GRAVITY_STANDARD_TREE));
    }
    if (c->prm.gravity_method == NCORP_GRAVITY_STANDARD_TREE) {
        PhaseTimer t(c, NCORP_PHASE_GWALK, s);
        HIPCHK(c, launch_standard_tree(ws, n, c->prm.p, c->prm.ncb_pre, c->prm.ncb_post, ax, ay,
                                       az, s));
        c->grav_lists = false;
        c->last = s;
        return NCORP_OK;
    }
    {
        PhaseTimer t(c, NCORP_PHASE_GWALK, s);
        ws.timing = c->timing;
        HIPCHK(c, launch_walk(ws, 0, c->prm.ncs, c->prm.ncc_pre, c->prm.ncc_post,
                              walk_waves(c->prm), s, &c->prm));
    }
    {
        PhaseTimer t(c, NCORP_PHASE_M2L, s);
        HIPCHK(c, launch_sort_long_lists(ws, s));
        HIPCHK(c, launch_m2l(ws, c->prm.p, c->prm.precision, s));
    }
    {
        PhaseTimer t(c, NCORP_PHASE_DESCENT, s);
        HIPCHK(c, launch_l2l(ws, c->prm.p, s));
    }
    {
        PhaseTimer t(c, NCORP_PHASE_P2P, s);
        HIPCHK(c, launch_p2p(ws, n, c->prm.precision, c->prm.p2p_tile, c->prm.p2p_targets_max,
                             s));
    }
    {
        PhaseTimer t(c, NCORP_PHASE_L2P, s);
        HIPCHK(c, launch_l2p(ws, n, c->prm.p, ax, ay, az, s, acc4));
    }
    if (c->timing) HIPCHK(c, launch_count_interactions(ws, s));
    c->grav_lists = true;
    c->last = s;
    return NCORP_OK;
}

extern "C" int ncorp_gravity(ncorp_ctx *c, const double *m, double *ax, double *ay, double *az,
                             void *stream) {
    if (!c) return NCORP_E_INVALID;
    if (mesh_gravity(c->prm) ? !c->have_mesh : !c->have_tree)
        return fail(c, NCORP_E_INVALID, mesh_gravity(c->prm)
                                            ? "no mesh: call ncorp_build_mesh first"
                                            : "no tree: call ncorp_build_tree first");
    if (!m || !ax || !ay || !az) return fail(c, NCORP_E_INVALID, "array pointer is NULL");
    return gravity_impl(c, m, ax, ay, az, (hipStream_t)stream);
}

// state: x, y, z, vx, vy, vz of a step (resolved in place when collisions are
// resolved), or nullptr for the search alone
static int collide_impl(ncorp_ctx *c, const double *vx, const double *vy, const double *vz,
                        const double *R, double dt, int64_t *pairs, int64_t cap,
                        int64_t *n_pairs_dev, int triple, int step, hipStream_t s,
                        double *const *state = nullptr, const double *m = nullptr) {
    // inside ncorp_step the kick before the search already wrote the packed (v, R)
    // records in input order
    const bool packed = state != nullptr;
    Workspace &ws = c->ws;
    const int64_t n = c->n;
    PhaseTimer t(c, NCORP_PHASE_COLLIDE, s);
    bool tree_tests = false;    // the tree's pair tests left per-block counts to add
    if (mesh_collisions(c->prm)) {
        HIPCHK(c, launch_mesh_collide(ws, vx, vy, vz, R, n, dt, !c->mesh_counted, s));
        c->mesh_counted = true;
    } else if (c->prm.collision_method == NCORP_COLLISIONS_BRUTE_FORCE) {
        if (ws.ndisks > 1)
            return fail(c, NCORP_E_UNSUPPORTED, "brute-force collisions take plain calls only");
        HIPCHK(c, launch_gather_vr(ws, packed, vx, vy, vz, R, n, s));
        HIPCHK(c, launch_collide_reset(ws, s));
        HIPCHK(c, launch_brute_collide(ws, n, dt, s));
    } else if (c->prm.collision_method == NCORP_COLLISIONS_STANDARD_TREE) {
        HIPCHK(c, launch_gather_vr(ws, packed, vx, vy, vz, R, n, s));
        {
            const bool reset = !ws.arrive_clean;
            ws.arrive_clean = false;
            HIPCHK(c, launch_collision_climb(ws, n, dt, s, reset));
        }
        HIPCHK(c, launch_collide_reset(ws, s));
        HIPCHK(c, launch_standard_tree_collide(ws, n, c->prm.ncb_pre, c->prm.ncb_post, dt, s));
    } else {
        tree_tests = true;
        if (c->grav_lists) {
            // candidates from the gravity walk's lists of this tree, culled with the
            // moonlets' bounding boxes (no collision climb needed); the box pass gathers
            // the packed (v, R) records itself
            if (!packed) HIPCHK(c, launch_pack_vr(ws, vx, vy, vz, R, n, s));
            HIPCHK(c, launch_leaf_boxes(ws, n, dt, s));
            HIPCHK(c, launch_candidates_from_lists(ws, s));
            HIPCHK(c, launch_collide_pairs(ws, n, dt, true, s));
        } else {
            HIPCHK(c, launch_gather_vr(ws, packed, vx, vy, vz, R, n, s));
            {
                const bool reset = !ws.arrive_clean;
                ws.arrive_clean = false;
                HIPCHK(c, launch_collision_climb(ws, n, dt, s, reset));
            }
            HIPCHK(c, launch_walk(ws, 1, c->prm.ncs_col, c->prm.ncc_pre_col,
                                  c->prm.ncc_post_col, 0, s));
            HIPCHK(c, launch_collide_pairs(ws, n, dt, false, s));
        }
    }
    if (state && c->prm.collision_mode == NCORP_COLLISIONS_RESOLVE)
        HIPCHK(c, launch_resolve(ws, state[0], state[1], state[2], state[3], state[4], state[5],
                                 m, R, dt, c->prm.collision_f, pairs, cap, n_pairs_dev, step,
                                 &ws.st->pair_cursor, tree_tests ? ws.count_part : nullptr,
                                 kCollideGrid, s));
    else
        HIPCHK(c, launch_emit_pairs(ws, pairs, cap, n_pairs_dev, triple, step,
                                    &ws.st->pair_cursor, tree_tests ? ws.count_part : nullptr,
                                    kCollideGrid, s));
    c->last = s;
    return NCORP_OK;
}

extern "C" int ncorp_collide(ncorp_ctx *c, const double *vx, const double *vy, const double *vz,
                             const double *R, double dt, int64_t *pairs, int64_t cap,
                             int64_t *n_pairs_dev, void *stream) {
    if (!c) return NCORP_E_INVALID;
    if (mesh_collisions(c->prm) ? !c->have_mesh : !c->have_tree)
        return fail(c, NCORP_E_INVALID, mesh_collisions(c->prm)
                                            ? "no mesh: call ncorp_build_mesh first"
                                            : "no tree: call ncorp_build_tree first");
    if (!vx || !vy || !vz || !R || !n_pairs_dev || (cap > 0 && !pairs))
        return fail(c, NCORP_E_INVALID, "array pointer is NULL");
    if (cap < 0) return fail(c, NCORP_E_INVALID, "cap must be >= 0");
    if (!(dt >= 0.0)) return fail(c, NCORP_E_INVALID, "dt must be >= 0");
    return collide_impl(c, vx, vy, vz, R, dt, pairs, cap, n_pairs_dev, 0, 0, (hipStream_t)stream);
}

namespace ncorp {
__global__ void k_zero_cursor(DevState *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->pair_cursor = 0;
}
}

// What the kick adds to the mutual gravity at time t: the central mass (App. B.1),
// the bulge of the central body and the quadrupolar tide of a distant body on a
// circular orbit (its position at t).
static CentralBody central_body(const ncorp_params &p, double t) {
    CentralBody b;
    b.GM = p.G * p.M_central;
    b.GMR2J2 = p.G * p.M_central * p.R_central * p.R_central * p.J2;
    b.GMsun = p.G * p.M_sun;
    b.sx = b.sy = b.sz = 0.0;
    b.a2 = b.a3 = 1.0;
    if (p.M_sun > 0.0) {
        const double a = p.a_sun;
        const double lam = t * std::sqrt(p.G * p.M_sun / (a * a * a));
        b.sx = a * std::cos(lam);
        b.sy = a * std::sin(lam) * std::cos(p.obliquity);
        b.sz = a * std::sin(lam) * std::sin(p.obliquity);
        b.a2 = a * a;
        b.a3 = a * a * a;
    }
    return b;
}

static int step_impl(ncorp_ctx *c, const int64_t *disk_off, int n_disks, double *x, double *y,
                     double *z, double *vx, double *vy, double *vz, const double *m,
                     const double *R, int64_t n, double dt, int n_steps, int64_t *pairs,
                     int64_t cap, int64_t *n_pairs_dev, void *workspace, int64_t ws_bytes,
                     void *stream) {
    if (!x || !y || !z || !vx || !vy || !vz || !m || !R || !n_pairs_dev || (cap > 0 && !pairs))
        return fail(c, NCORP_E_INVALID, "array pointer is NULL");
    if (n < 1 || n > INT32_MAX - 1) return fail(c, NCORP_E_INVALID, "n must be in 1..2^31-2");
    if (n_steps < 1) return fail(c, NCORP_E_INVALID, "n_steps must be >= 1");
    if (!(dt > 0.0)) return fail(c, NCORP_E_INVALID, "dt must be > 0");
    if (cap < 0) return fail(c, NCORP_E_INVALID, "cap must be >= 0");
    int r = setup_workspace(c, n, workspace, ws_bytes);
    if (r != NCORP_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    Workspace &ws = c->ws;
    double *ax = ws.acc, *ay = ws.acc + n, *az = ws.acc + 2 * n;
    const bool mutual = c->prm.p > 0;
    const bool need_mesh = (mutual && mesh_gravity(c->prm)) || mesh_collisions(c->prm);
    const bool need_tree = (mutual && !mesh_gravity(c->prm)) || !mesh_collisions(c->prm);
    if (need_mesh && disk_off)
        return fail(c, NCORP_E_UNSUPPORTED, "the mesh module takes plain (not batched) calls");
    // a plain tree build after the drift takes max |coordinate| from the drift
    const bool drift_max = need_tree && !disk_off;
    auto rebuild = [&](bool fresh) -> int {
        int q = NCORP_OK;
        if (need_tree && (q = build_tree_impl(c, x, y, z, n, s, fresh, disk_off, n_disks,
                                              mutual ? m : nullptr,
                                              !fresh && drift_max)) != NCORP_OK)
            return q;
        if (need_mesh) q = build_mesh_impl(c, x, y, z, R, n, s, fresh && !need_tree);
        return q;
    };
    if ((r = rebuild(true)) != NCORP_OK) return r;
    k_zero_cursor<<<1, 64, 0, s>>>(ws.st);
    // falcON evaluations hand the kick one (ax, ay, az, 0) record per moonlet: the
    // collision records' buffer is free from the evaluation to the kick after it (the
    // next search rewrites it)
    double4 *const acc4 = mutual && gravity_by_l2p(c->prm) ? ws.pcol : nullptr;
    // each evaluation follows a rebuild that brought G m into tree order
    if (mutual && (r = gravity_impl(c, m, ax, ay, az, s, true, acc4)) != NCORP_OK) return r;
    {
        PhaseTimer t(c, NCORP_PHASE_INTEGRATE, s);
        HIPCHK(c, launch_kick(vx, vy, vz, mutual ? ax : nullptr, ay, az, x, y, z, n, 0.5 * dt,
                              central_body(c->prm, c->clock), R, ws.pack4, s, acc4));
    }
    for (int k = 0; k < n_steps; k++) {
        double *const state[6] = {x, y, z, vx, vy, vz};
        r = collide_impl(c, vx, vy, vz, R, dt, pairs, cap, n_pairs_dev + k, 1, k, s, state, m);
        if (r != NCORP_OK) return r;
        {
            PhaseTimer t(c, NCORP_PHASE_INTEGRATE, s);
            HIPCHK(c, launch_drift(x, y, z, vx, vy, vz, n, dt, s, drift_max ? ws.st : nullptr));
        }
        if ((r = rebuild(false)) != NCORP_OK) return r;
        if (mutual && (r = gravity_impl(c, m, ax, ay, az, s, true, acc4)) != NCORP_OK) return r;
        const double h = (k == n_steps - 1) ? 0.5 * dt : dt;
        PhaseTimer t(c, NCORP_PHASE_INTEGRATE, s);
        HIPCHK(c, launch_kick(vx, vy, vz, mutual ? ax : nullptr, ay, az, x, y, z, n, h,
                              central_body(c->prm, c->clock + (double)(k + 1) * dt), R,
                              ws.pack4, s, acc4));
    }
    c->clock += (double)n_steps * dt;
    c->last = s;
    return NCORP_OK;
}

extern "C" int ncorp_step(ncorp_ctx *c, double *x, double *y, double *z, double *vx, double *vy,
                          double *vz, const double *m, const double *R, int64_t n, double dt,
                          int n_steps, int64_t *pairs, int64_t cap, int64_t *n_pairs_dev,
                          void *workspace, int64_t ws_bytes, void *stream) {
    if (!c) return NCORP_E_INVALID;
    return step_impl(c, nullptr, 1, x, y, z, vx, vy, vz, m, R, n, dt, n_steps, pairs, cap,
                     n_pairs_dev, workspace, ws_bytes, stream);
}

extern "C" int ncorp_step_batched(ncorp_ctx *c, const int64_t *disk_offsets, int n_disks,
                                  double *x, double *y, double *z, double *vx, double *vy,
                                  double *vz, const double *m, const double *R, int64_t n,
                                  double dt, int n_steps, int64_t *pairs, int64_t cap,
                                  int64_t *n_pairs_dev, void *workspace, int64_t ws_bytes,
                                  void *stream) {
    if (!c) return NCORP_E_INVALID;
    int r = check_disks(c, disk_offsets, n_disks);
    if (r != NCORP_OK) return r;
    return step_impl(c, disk_offsets, n_disks, x, y, z, vx, vy, vz, m, R, n, dt, n_steps, pairs,
                     cap, n_pairs_dev, workspace, ws_bytes, stream);
}

// ---------------------------------------------------------------- allocation-free form
// The workspace of ncorp_step_noalloc: a fixed array in the library's code object.
// Every GPU the library runs on holds its own copy, from the first use on that GPU
// until the process ends.  In host code `scratch` names a host-side stand-in, never
// the device memory: its device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[NCORP_STATIC_WORKSPACE_BYTES];

static constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices] = {};

static int scratch_of_current_device(ncorp_ctx *c, void **out) {
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices)
        return fail(c, NCORP_E_UNSUPPORTED, "allocation-free form: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255u) != 0)
            return fail(c, NCORP_E_HIP, "allocation-free form: scratch address not usable");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NCORP_OK;
}

extern "C" int ncorp_step_noalloc(ncorp_ctx *c, double *x, double *y, double *z, double *vx,
                                  double *vy, double *vz, const double *m, const double *R,
                                  int64_t n, double dt, int n_steps, int64_t *pairs, int64_t cap,
                                  int64_t *n_pairs_dev, void *stream) {
    if (!c) return NCORP_E_INVALID;
    // argument and size checks need no device: reject before anything touches the GPU
    if (!x || !y || !z || !vx || !vy || !vz || !m || !R || !n_pairs_dev || (cap > 0 && !pairs))
        return fail(c, NCORP_E_INVALID, "array pointer is NULL");
    if (n < 1 || n > INT32_MAX - 1) return fail(c, NCORP_E_INVALID, "n must be in 1..2^31-2");
    if (n_steps < 1) return fail(c, NCORP_E_INVALID, "n_steps must be >= 1");
    if (!(dt > 0.0)) return fail(c, NCORP_E_INVALID, "dt must be > 0");
    if (cap < 0) return fail(c, NCORP_E_INVALID, "cap must be >= 0");
    Workspace probe;
    const int64_t need = layout_workspace(probe, c->prm, n, 1);
    if (need > (int64_t)NCORP_STATIC_WORKSPACE_BYTES) {
        std::snprintf(c->err, sizeof(c->err),
                      "allocation-free form: n=%lld needs %lld workspace bytes, the fixed "
                      "array holds %lld",
                      (long long)n, (long long)need, (long long)NCORP_STATIC_WORKSPACE_BYTES);
        return NCORP_E_INVALID;
    }
    void *ws = nullptr;
    int r = scratch_of_current_device(c, &ws);
    if (r != NCORP_OK) return r;
    // Another call (of any context) may have used this GPU's array since this context
    // last did: forget every binding so the call starts from cleared device state
    // (status word, walk queue, mesh state), as on a new workspace.
    c->ws = Workspace{};
    c->mesh_init = false;
    c->have_mesh = false;
    c->have_tree = false;
    return step_impl(c, nullptr, 1, x, y, z, vx, vy, vz, m, R, n, dt, n_steps, pairs, cap,
                     n_pairs_dev, ws, (int64_t)NCORP_STATIC_WORKSPACE_BYTES, stream);
}

static int sync_state(ncorp_ctx *c, DevState &h) {
    if (!c->ws.base) return fail(c, NCORP_E_INVALID, "no workspace bound yet");
    HIPCHK(c, hipStreamSynchronize(c->last));
    HIPCHK(c, hipMemcpy(&h, c->ws.st, sizeof(DevState), hipMemcpyDeviceToHost));
    return NCORP_OK;
}

extern "C" int ncorp_get_status(ncorp_ctx *c, int64_t *required) {
    if (!c) return NCORP_E_INVALID;
    DevState h;
    int r = sync_state(c, h);
    if (r != NCORP_OK) return r;
    if (required) *required = h.required;
    if (h.status & (ST_CAP_CELLS | ST_CAP_QUEUE | ST_CAP_M2L | ST_CAP_P2P | ST_CAP_PAIRS |
                    ST_CAP_LISTS | ST_CAP_MESH)) {
        std::snprintf(c->err, sizeof(c->err), "device list overflow (flags 0x%x, required %lld)",
                      h.status, (long long)h.required);
        return NCORP_E_CAPACITY;
    }
    if (h.status & (ST_WALK_STALL | ST_BAD_ITEM)) {
        std::snprintf(c->err, sizeof(c->err), "a tree pass stopped waiting (flags 0x%x)", h.status);
        return NCORP_E_HIP;
    }
    if (h.status & ST_BAD_OFFSETS)
        return fail(c, NCORP_E_INVALID, "disk offsets are not a non-decreasing 0..n sequence");
    if (h.status & ST_MESH_RANGE)
        return fail(c, NCORP_E_INVALID,
                    "mesh: a cell coordinate beyond 2^30 or a mesh size that is not > 0");
    if (h.status & ST_NONFINITE) return fail(c, NCORP_E_NONFINITE, "non-finite position");
    return NCORP_OK;
}

extern "C" int ncorp_tree_info(ncorp_ctx *c, int64_t *info) {
    if (!c || !info) return NCORP_E_INVALID;
    DevState h;
    int r = sync_state(c, h);
    if (r != NCORP_OK) return r;
    info[NCORP_INFO_N] = c->n;
    info[NCORP_INFO_NCELLS] = h.ncells;
    info[NCORP_INFO_NLEAVES] = h.nleaves;
    info[NCORP_INFO_MAXLEVEL] = h.maxlevel;
    info[NCORP_INFO_M2L] = h.nm2l;
    info[NCORP_INFO_P2P] = h.np2p;
    info[NCORP_INFO_VISITED] = h.visited;
    info[NCORP_INFO_COL_CAND] = h.ncand;
    info[NCORP_INFO_COL_TESTS] = h.col_tests;
    info[NCORP_INFO_M2L_DIR] = 2 * (int64_t)h.nm2l;
    info[NCORP_INFO_NROOTS] = h.level_count[0];
    info[NCORP_INFO_LONG_M2L] = h.nlong_m2l;
    info[NCORP_INFO_LONG_P2P] = h.nlong_p2p;
    info[NCORP_INFO_P2P_INTER] = h.p2p_inter;
    info[NCORP_INFO_M2L_MAXLIST] = h.m2l_maxlist;
    info[NCORP_INFO_P2P_MAXLIST] = h.p2p_maxlist;
    info[NCORP_INFO_WALK_BUSY_MAX] = h.walk_busy_max;
    info[NCORP_INFO_WALK_BUSY_MEAN] = h.walk_busy_sum / walk_waves(c->prm);
    info[NCORP_INFO_P2P_SRC_MAX] = h.p2p_src_max;
    info[NCORP_INFO_SORT_PREV] = h.bs_prev_used;
    info[NCORP_INFO_SORT_SPILL] = h.bs_spill;
    return NCORP_OK;
}

extern "C" int ncorp_set_timing(ncorp_ctx *c, int enable) {
    if (!c) return NCORP_E_INVALID;
    c->timing = enable != 0;
    return NCORP_OK;
}

extern "C" int ncorp_phase_times(ncorp_ctx *c, double *ms, int64_t *count) {
    if (!c) return NCORP_E_INVALID;
    for (auto &r : c->recs) {
        HIPCHK(c, hipEventSynchronize(r.b));
        float t = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&t, r.a, r.b));
        if (r.phase >= 0 && r.phase < NCORP_PHASE_COUNT) {
            if (ms) ms[r.phase] += (double)t;
            if (count) count[r.phase] += 1;
        }
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    return NCORP_OK;
}

template <typename T>
static int d2h(ncorp_ctx *c, std::vector<T> &v, const T *src, int64_t count) {
    v.resize(count > 0 ? count : 0);
    if (count > 0) HIPCHK(c, hipMemcpy(v.data(), src, sizeof(T) * count, hipMemcpyDeviceToHost));
    return NCORP_OK;
}

extern "C" int64_t ncorp_export_host(ncorp_ctx *c, int what, void *dst, int64_t bytes) {
    if (!c || bytes < 0 || (bytes > 0 && !dst)) return NCORP_E_INVALID;
    DevState h;
    int r = sync_state(c, h);
    if (r != NCORP_OK) return r;
    const Workspace &ws = c->ws;
    const int64_t n = c->n, nc = h.ncells;
    std::vector<char> out;
    auto put = [&](const void *p, int64_t b) {
        out.resize(b);
        if (b) std::memcpy(out.data(), p, b);
    };
    switch (what) {
        case NCORP_EXPORT_KEYS: {
            std::vector<uint64_t> v; if ((r = d2h(c, v, ws.keys, n))) return r;
            put(v.data(), 8 * n); break;
        }
        case NCORP_EXPORT_PERM: {
            std::vector<uint32_t> v; if ((r = d2h(c, v, ws.idx, n))) return r;
            put(v.data(), 4 * n); break;
        }
        case NCORP_EXPORT_CELLS: {
            std::vector<int32_t> lv, f, cn, ch, nch, par;
            std::vector<uint64_t> pre;
            if ((r = d2h(c, lv, ws.c_level, nc)) || (r = d2h(c, f, ws.c_first, nc)) ||
                (r = d2h(c, cn, ws.c_count, nc)) || (r = d2h(c, ch, ws.c_child, nc)) ||
                (r = d2h(c, nch, ws.c_nchild, nc)) || (r = d2h(c, par, ws.c_parent, nc)) ||
                (r = d2h(c, pre, ws.c_prefix, nc)))
                return r;
            std::vector<int32_t> v(8 * nc);
            for (int64_t i = 0; i < nc; i++) {
                v[8 * i + 0] = lv[i]; v[8 * i + 1] = f[i]; v[8 * i + 2] = cn[i];
                v[8 * i + 3] = ch[i]; v[8 * i + 4] = nch[i]; v[8 * i + 5] = par[i];
                v[8 * i + 6] = (int32_t)(pre[i] & 0xffffffffull);
                v[8 * i + 7] = (int32_t)(pre[i] >> 32);
            }
            put(v.data(), 4 * 8 * nc); break;
        }
        case NCORP_EXPORT_GCELLS: {
            std::vector<double4> g; std::vector<double> ms, rm, th;
            if ((r = d2h(c, g, ws.gcell, nc)) || (r = d2h(c, ms, ws.c_mass, nc)) ||
                (r = d2h(c, rm, ws.c_rmax, nc)) || (r = d2h(c, th, ws.c_theta, nc)))
                return r;
            std::vector<double> v(8 * nc);
            for (int64_t i = 0; i < nc; i++) {
                v[8 * i + 0] = g[i].x; v[8 * i + 1] = g[i].y; v[8 * i + 2] = g[i].z;
                v[8 * i + 3] = ms[i]; v[8 * i + 4] = rm[i]; v[8 * i + 5] = g[i].w;
                v[8 * i + 6] = th[i]; v[8 * i + 7] = 0.0;
            }
            put(v.data(), 8 * 8 * nc); break;
        }
        case NCORP_EXPORT_CCELLS: {
            std::vector<double4> g; std::vector<double> rm;
            if ((r = d2h(c, g, ws.ccell, nc)) || (r = d2h(c, rm, ws.c_crmax, nc))) return r;
            std::vector<double> v(5 * nc);
            for (int64_t i = 0; i < nc; i++) {
                v[4 * i + 0] = g[i].x; v[4 * i + 1] = g[i].y; v[4 * i + 2] = g[i].z;
                v[4 * i + 3] = g[i].w;
                v[4 * nc + i] = rm[i];
            }
            put(v.data(), 8 * 5 * nc); break;
        }
        case NCORP_EXPORT_MULTIPOLES: {
            std::vector<double> v; if ((r = d2h(c, v, ws.mult, nc * ws.nm))) return r;
            put(v.data(), 8 * nc * ws.nm); break;
        }
        case NCORP_EXPORT_LOCAL: {
            std::vector<double> v; if ((r = d2h(c, v, ws.local, nc * ws.nl))) return r;
            put(v.data(), 8 * nc * ws.nl); break;
        }
        case NCORP_EXPORT_M2L:
        case NCORP_EXPORT_P2P:
        case NCORP_EXPORT_COL_CAND: {
            // copy the reserved slots and drop the gaps
            const int2 *src = what == NCORP_EXPORT_M2L ? ws.m2l
                              : what == NCORP_EXPORT_P2P ? ws.p2p : ws.cand;
            const int64_t slots = what == NCORP_EXPORT_M2L ? h.m2l_slots
                                  : what == NCORP_EXPORT_P2P ? h.p2p_slots : h.cand_slots;
            const int64_t lcap = what == NCORP_EXPORT_M2L ? ws.m2l_cap : ws.p2p_cap;
            std::vector<int2> v;
            if ((r = d2h(c, v, src, slots < lcap ? slots : lcap))) return r;
            std::vector<int2> keep;
            keep.reserve(v.size());
            for (const int2 &q : v)
                if (q.x >= 0) keep.push_back(q);
            put(keep.data(), 8 * (int64_t)keep.size()); break;
        }
        default:
            return fail(c, NCORP_E_INVALID, "unknown export");
    }
    int64_t full = (int64_t)out.size();
    int64_t cp = full < bytes ? full : bytes;
    if (cp > 0) std::memcpy(dst, out.data(), cp);
    return full;
}

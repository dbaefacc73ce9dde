/*
 * ncorp_oracle.c -- plain, slow, FP64 CPU reference ("oracle") for the falcON
 * tree step of NcorpiON (Couturier, Quillen & Nakajima, "NcorpiON: A O(N)
 * software for N-body integration in collisional and fragmenting systems").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load or call this file.  It shares no code,
 * header, table or helper with the GPU library, and the GPU library never calls it.
 *
 * What is here, each following the passage named beside it:
 *   - pair collision test ............................ Sect. 3.1, Eqs. (1)-(2)
 *   - root cube and 3-D Hilbert keys ................. Sect. 3.4.6 (Skilling's
 *                                                       transpose form; reading)
 *   - pointer octree by insertion, flattened ......... Sect. 3.4.1, Sect. 3.4.6
 *   - derivative tensors of 1/R ...................... Eq. (17), by jet arithmetic
 *   - inner / outer products on full 3^n tensors ..... Eqs. (18)-(19)
 *   - gravity climb .................................. Eqs. (10)-(12), corner clamp,
 *                                                       multipoles by Eq. (20)
 *   - TreeWalk ....................................... Alg. 2 (falcON walk)
 *   - M2L interaction tensors ........................ Eq. (25), both directions
 *   - tree descent and evaluation .................... Eq. (26)
 *   - collision climb + walk ......................... Eqs. (7)-(9), Alg. 2
 *   - direct sum (Neumaier compensated) and brute-force pair scan (Sect. 3.2)
 *   - grid-filtered pair scan, exactly the brute-force set ... Sect. 3.1
 *
 * Tensors are kept in full 3^n form with index i1*3^(n-1)+...+in, so nothing
 * here depends on the symmetric storage the GPU uses.  Multipole moments are
 * taken straight from their definition (Eq. 20) at every cell; the shift
 * formulas of the appendix are not used here.  The walk is recursive, exactly
 * as printed.  Readings where the paper is silent:
 *   R1 root cube centred on the central mass, half-width the smallest power of
 *      two strictly larger than every |coordinate|;
 *   R2 q = floor((x+L) * 2^20 / L) per axis, clamped to [0, 2^21-1]; Hilbert key
 *      = Skilling transpose of (qx,qy,qz), bits interleaved x,y,z from the top;
 *   R3 theta(M): theta^5/(1-theta)^2 = theta_min^5/(1-theta_min)^2 (M/M_root)^(-1/3),
 *      solved (cubed, so only + - * / are used) by 64 bisection steps;
 *   R4 maximum depth 21; R5 a cell with count <= s is a leaf;
 *   R6 moonlets inside a leaf ordered by (key, input index);
 *   R7 collision centre = unweighted centroid of the cell's moonlets (Eq. 7 with
 *      child weights n_a);
 *   R8 corner clamp at every cell, parents use the clamped value;
 *   R9 thresholds exactly as printed ("<=" for N_cs, "<" for N_cc, MAC "<=");
 *   R10 split A iff B is a leaf or (A is not a leaf and r_crit,A > r_crit,B);
 *   R11 self pair -> all unordered child pairs (a <= b), including (a, a);
 *   R12 no softening, j == i skipped;  R16 dv^2 = 0 or Delta < 0 -> no collision;
 *   R18 p = 0 -> no mutual gravity; M^(1) vanishes at the centre of mass and is
 *      not used, M^(p) and C^(0) are never formed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXDEPTH 21
#define ORC_MAXP 6

static int ipow3(int n) { int r = 1; while (n-- > 0) r *= 3; return r; }

/* ------------------------------------------------------------------------- */
/* Pair collision test, Sect. 3.1 Eqs. (1)-(2).  1 iff the straight-line       */
/* trajectories bring the spheres into contact at a time 0 <= dt_c <= dt.      */
/* ------------------------------------------------------------------------- */
int orc_pair_test(double x1, double y1, double z1, double vx1, double vy1, double vz1,
                  double R1, double x2, double y2, double z2, double vx2, double vy2,
                  double vz2, double R2, double dt)
{
    double dx = x1 - x2, dy = y1 - y2, dz = z1 - z2;
    double dvx = vx1 - vx2, dvy = vy1 - vy2, dvz = vz1 - vz2;
    double rv = dx * dvx + dy * dvy + dz * dvz;
    double v2 = dvx * dvx + dvy * dvy + dvz * dvz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double Rs = R1 + R2;
    double disc = rv * rv + v2 * (Rs * Rs - r2);          /* Eq. (1) */
    if (!(v2 > 0.0) || !(disc >= 0.0)) return 0;
    double tc = -(rv + sqrt(disc)) / v2;                   /* Eq. (2) */
    return (tc >= 0.0 && tc <= dt) ? 1 : 0;
}

/* Time of contact dt_c of Eq. (2) when 0 <= dt_c <= dt, else -1. */
double orc_collision_time(double x1, double y1, double z1, double vx1, double vy1, double vz1,
                          double R1, double x2, double y2, double z2, double vx2, double vy2,
                          double vz2, double R2, double dt)
{
    double dx = x1 - x2, dy = y1 - y2, dz = z1 - z2;
    double dvx = vx1 - vx2, dvy = vy1 - vy2, dvz = vz1 - vz2;
    double rv = dx * dvx + dy * dvy + dz * dvz;
    double v2 = dvx * dvx + dvy * dvy + dvz * dvz;
    double r2 = dx * dx + dy * dy + dz * dz;
    double Rs = R1 + R2;
    double disc = rv * rv + v2 * (Rs * Rs - r2);
    if (!(v2 > 0.0) || !(disc >= 0.0)) return -1.0;
    double tc = -(rv + sqrt(disc)) / v2;
    return (tc >= 0.0 && tc <= dt) ? tc : -1.0;
}

/* ------------------------------------------------------------------------- */
/* Collision resolution, Sect. 5.1 and 5.2 (the order rule below is a reading: */
/* the paper gives none).                                                      */
/* The colliding pairs (i < j, one row each) are taken in increasing order of  */
/* (dt_c, i, j); a pair is resolved unless one of its moonlets already was in  */
/* this step.  Resolving (1 = i, 2 = j): both move on straight lines to the    */
/* contact time dt_c, dr = r1 - r2 and dv = v1 - v2 there, the impulse          */
/*   J = alpha (dr . dv) dr,  alpha = f m1 m2 / ((m1 + m2) (R1 + R2)^2)         */
/* changes v1 by -J/m1 and v2 by +J/m2 (f = 2: elastic), and the rest of the    */
/* drift uses the new velocity.  The state given is (r, v) at the start of the */
/* drift; on return v holds v' and r holds r + dt_c (v - v'), so that the      */
/* drift r + dt v' that follows lands where the moonlet ends the step.         */
/* resolved[k] = 1 for the pairs resolved.  Returns their number.              */
/* ------------------------------------------------------------------------- */
typedef struct { double t; int64_t i, j, k; } orc_hit;

static int hit_cmp(const void *a, const void *b)
{
    const orc_hit *p = (const orc_hit *)a, *q = (const orc_hit *)b;
    if (p->t != q->t) return p->t < q->t ? -1 : 1;
    if (p->i != q->i) return p->i < q->i ? -1 : 1;
    if (p->j != q->j) return p->j < q->j ? -1 : 1;
    return 0;
}

int64_t orc_resolve(int64_t npairs, const int64_t *pairs, int64_t n, double *x, double *y,
                    double *z, double *vx, double *vy, double *vz, const double *m,
                    const double *R, double dt, double f, int32_t *resolved)
{
    orc_hit *h = (orc_hit *)malloc(sizeof(orc_hit) * (size_t)(npairs > 0 ? npairs : 1));
    char *used = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int64_t nh = 0, nres = 0;
    for (int64_t k = 0; k < npairs; k++) {
        int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
        resolved[k] = 0;
        double t = orc_collision_time(x[i], y[i], z[i], vx[i], vy[i], vz[i], R[i], x[j], y[j],
                                      z[j], vx[j], vy[j], vz[j], R[j], dt);
        if (t < 0.0) continue;            /* not a collision of this step */
        h[nh].t = t; h[nh].i = i; h[nh].j = j; h[nh].k = k;
        nh++;
    }
    qsort(h, (size_t)nh, sizeof(orc_hit), hit_cmp);
    for (int64_t q = 0; q < nh; q++) {
        int64_t i = h[q].i, j = h[q].j;
        if (used[i] || used[j]) continue;
        used[i] = used[j] = 1;
        resolved[h[q].k] = 1;
        nres++;
        double t = h[q].t;
        double x1 = x[i] + t * vx[i], y1 = y[i] + t * vy[i], z1 = z[i] + t * vz[i];
        double x2 = x[j] + t * vx[j], y2 = y[j] + t * vy[j], z2 = z[j] + t * vz[j];
        double drx = x1 - x2, dry = y1 - y2, drz = z1 - z2;
        double dvx = vx[i] - vx[j], dvy = vy[i] - vy[j], dvz = vz[i] - vz[j];
        double s = drx * dvx + dry * dvy + drz * dvz;
        double Rs = R[i] + R[j];
        double alpha = f * m[i] * m[j] / ((m[i] + m[j]) * (Rs * Rs));
        double Jx = alpha * s * drx, Jy = alpha * s * dry, Jz = alpha * s * drz;
        double u1x = vx[i] - Jx / m[i], u1y = vy[i] - Jy / m[i], u1z = vz[i] - Jz / m[i];
        double u2x = vx[j] + Jx / m[j], u2y = vy[j] + Jy / m[j], u2z = vz[j] + Jz / m[j];
        x[i] = x[i] + t * (vx[i] - u1x); y[i] = y[i] + t * (vy[i] - u1y);
        z[i] = z[i] + t * (vz[i] - u1z);
        x[j] = x[j] + t * (vx[j] - u2x); y[j] = y[j] + t * (vy[j] - u2y);
        z[j] = z[j] + t * (vz[j] - u2z);
        vx[i] = u1x; vy[i] = u1y; vz[i] = u1z;
        vx[j] = u2x; vy[j] = u2y; vz[j] = u2z;
    }
    free(h);
    free(used);
    return nres;
}

/* ------------------------------------------------------------------------- */
/* Root cube and Hilbert keys (Sect. 3.4.6; readings R1, R2).                  */
/* ------------------------------------------------------------------------- */
double orc_root_half_width(const double *x, const double *y, const double *z, int64_t n)
{
    double mx = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double a = fabs(x[i]), b = fabs(y[i]), c = fabs(z[i]);
        if (a > mx) mx = a;
        if (b > mx) mx = b;
        if (c > mx) mx = c;
    }
    /* smallest power of two strictly above mx (1 for an all-zero input) */
    if (!(mx > 0.0)) return 1.0;
    double L = 1.0;
    while (L <= mx) L *= 2.0;
    while (L * 0.5 > mx) L *= 0.5;
    return L;
}

uint32_t orc_quantize(double x, double L)
{
    double t = (x + L) * (1048576.0 / L);
    if (!(t >= 0.0)) return 0u;
    if (t >= 2097152.0) return 2097151u;
    uint32_t q = (uint32_t)floor(t);
    return q > 2097151u ? 2097151u : q;
}

/* Hilbert index of a point with integer coordinates X[0..2], `bits` bits each,
 * following Skilling ("Programming the Hilbert curve", AIP Conf. Proc. 707,
 * 2004): undo the excess work of the inverse transform level by level, Gray-
 * encode, then read the transposed bits out from the top, x then y then z. */
uint64_t orc_hilbert_index(uint32_t X0, uint32_t X1, uint32_t X2, int bits)
{
    uint32_t X[3] = {X0, X1, X2};
    uint32_t top = 1u << (bits - 1);
    for (uint32_t Q = top; Q > 1u; Q >>= 1) {
        uint32_t P = Q - 1u;
        for (int i = 0; i < 3; i++) {
            if (X[i] & Q) {
                X[0] ^= P;                        /* invert low bits of X[0] */
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;   /* swap low bits of X[0], X[i] */
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = top; Q > 1u; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1u;
    X[0] ^= t; X[1] ^= t; X[2] ^= t;
    uint64_t h = 0;
    for (int b = bits - 1; b >= 0; b--)
        for (int i = 0; i < 3; i++)
            h = (h << 1) | (uint64_t)((X[i] >> b) & 1u);
    return h;
}

void orc_hilbert_keys(const double *x, const double *y, const double *z, int64_t n,
                      double L, uint64_t *keys)
{
    for (int64_t i = 0; i < n; i++)
        keys[i] = orc_hilbert_index(orc_quantize(x[i], L), orc_quantize(y[i], L),
                                    orc_quantize(z[i], L), ORC_MAXDEPTH);
}

/* ------------------------------------------------------------------------- */
/* Pointer octree built by insertion (Sect. 3.4.1: cells with at most s       */
/* moonlets are not divided), then copied into a flat array ordered by level,  */
/* then Hilbert order inside a level, children contiguous (Sect. 3.4.6).       */
/* ------------------------------------------------------------------------- */
typedef struct onode {
    int level;
    uint32_t cx, cy, cz;          /* integer cube coordinates at this level */
    int64_t n;                    /* moonlets inside */
    int64_t *ids, cap;            /* moonlet ids while a leaf */
    struct onode *child[8];
    int leaf;
    int64_t flat;                 /* index in the flat tree */
} onode;

typedef struct orc_tree {
    int64_t n, ncells;
    int s;
    double L;
    uint64_t *keys;               /* per input moonlet */
    uint32_t *q;                  /* quantized coordinates, 3 per moonlet */
    int64_t *perm;                /* tree order position -> input index */
    int32_t *level, *first, *count, *child_first, *nchild, *parent;
    uint32_t *cx, *cy, *cz;
    uint64_t *prefix;
    int maxlevel;
} orc_tree;

static onode *node_new(int level, uint32_t cx, uint32_t cy, uint32_t cz)
{
    onode *nd = (onode *)calloc(1, sizeof(onode));
    nd->level = level; nd->cx = cx; nd->cy = cy; nd->cz = cz;
    nd->leaf = 1;
    return nd;
}

static void node_insert(onode *nd, int64_t id, const uint32_t *q, int s);

static void node_route(onode *nd, int64_t id, const uint32_t *q, int s)
{
    int sh = ORC_MAXDEPTH - 1 - nd->level;   /* bit selecting the child octant */
    int bx = (q[3 * id + 0] >> sh) & 1, by = (q[3 * id + 1] >> sh) & 1,
        bz = (q[3 * id + 2] >> sh) & 1;
    int o = bx * 4 + by * 2 + bz;
    if (!nd->child[o])
        nd->child[o] = node_new(nd->level + 1, 2 * nd->cx + bx, 2 * nd->cy + by,
                                2 * nd->cz + bz);
    node_insert(nd->child[o], id, q, s);
}

static void node_insert(onode *nd, int64_t id, const uint32_t *q, int s)
{
    nd->n++;
    if (!nd->leaf) { node_route(nd, id, q, s); return; }
    if (nd->n > nd->cap) {
        nd->cap = nd->cap ? 2 * nd->cap : 8;
        nd->ids = (int64_t *)realloc(nd->ids, (size_t)nd->cap * sizeof(int64_t));
    }
    nd->ids[nd->n - 1] = id;
    if (nd->n > s && nd->level < ORC_MAXDEPTH) {
        int64_t *ids = nd->ids, m = nd->n;
        nd->ids = NULL; nd->cap = 0; nd->leaf = 0; nd->n = 0;
        for (int64_t k = 0; k < m; k++) { nd->n++; node_route(nd, ids[k], q, s); }
        free(ids);
    }
}

static void node_free(onode *nd)
{
    if (!nd) return;
    for (int o = 0; o < 8; o++) node_free(nd->child[o]);
    free(nd->ids);
    free(nd);
}

static const uint64_t *g_sort_keys;
static int cmp_key_id(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    uint64_t ki = g_sort_keys[i], kj = g_sort_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

/* Hilbert position of a cell = key of any of its moonlets cut to its level. */
static uint64_t node_prefix(const onode *nd, const uint64_t *keys)
{
    const onode *c = nd;
    while (!c->leaf) {
        for (int o = 0; o < 8; o++) if (c->child[o]) { c = c->child[o]; break; }
    }
    return keys[c->ids[0]] >> (3 * (ORC_MAXDEPTH - nd->level));
}

static int cmp_child(const void *a, const void *b)
{
    uint64_t pa = ((const uint64_t *)a)[0], pb = ((const uint64_t *)b)[0];
    return pa < pb ? -1 : (pa > pb ? 1 : 0);
}

/* Children of nd, sorted along the Hilbert curve. */
static int sorted_children(const onode *nd, const uint64_t *keys, onode **out)
{
    uint64_t tmp[8][2];
    int k = 0;
    for (int o = 0; o < 8; o++)
        if (nd->child[o]) {
            tmp[k][0] = node_prefix(nd->child[o], keys);
            tmp[k][1] = (uint64_t)(uintptr_t)nd->child[o];
            k++;
        }
    qsort(tmp, (size_t)k, sizeof(tmp[0]), cmp_child);
    for (int i = 0; i < k; i++) out[i] = (onode *)(uintptr_t)tmp[i][1];
    return k;
}

static void assign_particles(onode *nd, const uint64_t *keys, int64_t *perm,
                             int64_t *pos, int64_t *firstpos)
{
    firstpos[nd->flat] = *pos;
    if (nd->leaf) {
        g_sort_keys = keys;
        qsort(nd->ids, (size_t)nd->n, sizeof(int64_t), cmp_key_id);
        for (int64_t k = 0; k < nd->n; k++) perm[(*pos)++] = nd->ids[k];
        return;
    }
    onode *ch[8];
    int k = sorted_children(nd, keys, ch);
    for (int i = 0; i < k; i++) assign_particles(ch[i], keys, perm, pos, firstpos);
}

orc_tree *orc_tree_build(const double *x, const double *y, const double *z, int64_t n,
                         double L, int s)
{
    if (n <= 0 || s < 1) return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->n = n; t->s = s; t->L = L;
    t->keys = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    t->q = (uint32_t *)malloc((size_t)n * 3 * sizeof(uint32_t));
    for (int64_t i = 0; i < n; i++) {
        t->q[3 * i + 0] = orc_quantize(x[i], L);
        t->q[3 * i + 1] = orc_quantize(y[i], L);
        t->q[3 * i + 2] = orc_quantize(z[i], L);
        t->keys[i] = orc_hilbert_index(t->q[3 * i], t->q[3 * i + 1], t->q[3 * i + 2],
                                       ORC_MAXDEPTH);
    }
    onode *root = node_new(0, 0, 0, 0);
    for (int64_t i = 0; i < n; i++) node_insert(root, i, t->q, s);

    /* breadth-first flattening, children appended in Hilbert order */
    int64_t cap = 1024, head = 0, tail = 0;
    onode **queue = (onode **)malloc((size_t)cap * sizeof(onode *));
    queue[tail++] = root;
    while (head < tail) {
        onode *nd = queue[head];
        nd->flat = head++;
        if (nd->leaf) continue;
        onode *ch[8];
        int k = sorted_children(nd, t->keys, ch);
        for (int i = 0; i < k; i++) {
            if (tail == cap) {
                cap *= 2;
                queue = (onode **)realloc(queue, (size_t)cap * sizeof(onode *));
            }
            queue[tail++] = ch[i];
        }
    }
    int64_t nc = tail;
    t->ncells = nc;
    t->level = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    t->first = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    t->count = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    t->child_first = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    t->nchild = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    t->parent = (int32_t *)malloc((size_t)nc * sizeof(int32_t));
    t->cx = (uint32_t *)malloc((size_t)nc * sizeof(uint32_t));
    t->cy = (uint32_t *)malloc((size_t)nc * sizeof(uint32_t));
    t->cz = (uint32_t *)malloc((size_t)nc * sizeof(uint32_t));
    t->prefix = (uint64_t *)malloc((size_t)nc * sizeof(uint64_t));
    t->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *firstpos = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
    int64_t pos = 0;
    assign_particles(root, t->keys, t->perm, &pos, firstpos);
    t->maxlevel = 0;
    t->parent[0] = -1;
    for (int64_t c = 0; c < nc; c++) {
        onode *nd = queue[c];
        t->level[c] = nd->level;
        if (nd->level > t->maxlevel) t->maxlevel = nd->level;
        t->first[c] = (int32_t)firstpos[c];
        t->count[c] = (int32_t)nd->n;
        t->cx[c] = nd->cx; t->cy[c] = nd->cy; t->cz[c] = nd->cz;
        t->prefix[c] = node_prefix(nd, t->keys);
        if (nd->leaf) { t->child_first[c] = -1; t->nchild[c] = 0; continue; }
        onode *ch[8];
        int k = sorted_children(nd, t->keys, ch);
        t->child_first[c] = (int32_t)ch[0]->flat;
        t->nchild[c] = k;
        for (int i = 0; i < k; i++) t->parent[ch[i]->flat] = (int32_t)c;
    }
    free(firstpos);
    free(queue);
    node_free(root);
    return t;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->keys); free(t->q); free(t->perm);
    free(t->level); free(t->first); free(t->count); free(t->child_first);
    free(t->nchild); free(t->parent); free(t->cx); free(t->cy); free(t->cz);
    free(t->prefix);
    free(t);
}

int64_t orc_tree_ncells(const orc_tree *t) { return t->ncells; }
int orc_tree_maxlevel(const orc_tree *t) { return t->maxlevel; }

void orc_tree_export(const orc_tree *t, int32_t *level, int32_t *first, int32_t *count,
                     int32_t *child_first, int32_t *nchild, int32_t *parent,
                     uint64_t *prefix, int64_t *perm, uint64_t *keys)
{
    int64_t nc = t->ncells;
    memcpy(level, t->level, (size_t)nc * 4);
    memcpy(first, t->first, (size_t)nc * 4);
    memcpy(count, t->count, (size_t)nc * 4);
    memcpy(child_first, t->child_first, (size_t)nc * 4);
    memcpy(nchild, t->nchild, (size_t)nc * 4);
    memcpy(parent, t->parent, (size_t)nc * 4);
    memcpy(prefix, t->prefix, (size_t)nc * 8);
    memcpy(perm, t->perm, (size_t)t->n * 8);
    memcpy(keys, t->keys, (size_t)t->n * 8);
}

/* Geometric cube of a cell: centre and half-width (exact in FP64). */
static void cell_cube(const orc_tree *t, int64_t c, double cen[3], double *h)
{
    int lv = t->level[c];
    double hw = ldexp(t->L, -lv);
    double side = ldexp(1.0, lv);
    cen[0] = hw * (2.0 * (double)t->cx[c] + 1.0 - side);
    cen[1] = hw * (2.0 * (double)t->cy[c] + 1.0 - side);
    cen[2] = hw * (2.0 * (double)t->cz[c] + 1.0 - side);
    *h = hw;
}

/* Distance from point s to the farthest corner of the cell's cube (Sect. 3.4.2). */
static double far_corner(const orc_tree *t, int64_t c, const double s[3])
{
    double cen[3], h;
    cell_cube(t, c, cen, &h);
    double dx = fabs(s[0] - cen[0]) + h;
    double dy = fabs(s[1] - cen[1]) + h;
    double dz = fabs(s[2] - cen[2]) + h;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

static double dist3(const double a[3], const double b[3])
{
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Reading R3 of Dehnen's mass-dependent opening angle, with the cube root moved
 * to the other side so that only correctly rounded + - * / are used:
 *   theta^15 * M = K^3 * M_root * (1 - theta)^6,  K = theta_min^5/(1-theta_min)^2. */
double orc_theta_of_mass(double M, double M_root, double theta_min)
{
    if (!(M < M_root)) return theta_min;
    double tm = theta_min, um = 1.0 - theta_min;
    double tm2 = tm * tm, tm4 = tm2 * tm2, tm5 = tm4 * tm;
    double um2 = um * um;
    double K = tm5 / um2;
    double K3 = K * K * K;
    double rhs0 = K3 * M_root;
    double lo = theta_min, hi = 1.0;
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (lo + hi);
        double t2 = mid * mid, t4 = t2 * t2, t8 = t4 * t4;
        double t15 = t8 * t4 * t2 * mid;
        double u = 1.0 - mid, u2 = u * u, u4 = u2 * u2, u6 = u4 * u2;
        double g = t15 * M - rhs0 * u6;
        if (g <= 0.0) lo = mid; else hi = mid;
    }
    return lo;
}

/* ------------------------------------------------------------------------- */
/* Derivative tensors of g(R) = 1/|R| (Eq. 17) by jet arithmetic:              */
/*   1/|R+h| = r^-1 (1+u)^(-1/2),  u = (2 R.h + h.h)/r^2,                      */
/* expanded with the binomial series to total degree n in h.  The coefficient  */
/* of h^a (a = exponents along x, y, z) is D_a / a!, D_a = d^a g(R).           */
/* ------------------------------------------------------------------------- */
#define JD (ORC_MAXP + 1)
typedef double jet_t[JD][JD][JD];

static void jet_zero(jet_t j) { memset(j, 0, sizeof(jet_t)); }

/* out = a * u  truncated at total degree nmax; u has the linear terms ul[3]
 * and the squares uq (same coefficient for x^2, y^2, z^2). */
static void jet_mul_u(jet_t out, jet_t a, const double ul[3], double uq, int nmax)
{
    jet_zero(out);
    for (int i = 0; i <= nmax; i++)
        for (int j = 0; i + j <= nmax; j++)
            for (int k = 0; i + j + k <= nmax; k++) {
                double c = a[i][j][k];
                if (c == 0.0) continue;
                int d = i + j + k;
                if (d + 1 <= nmax) {
                    out[i + 1][j][k] += c * ul[0];
                    out[i][j + 1][k] += c * ul[1];
                    out[i][j][k + 1] += c * ul[2];
                }
                if (d + 2 <= nmax) {
                    out[i + 2][j][k] += c * uq;
                    out[i][j + 2][k] += c * uq;
                    out[i][j][k + 2] += c * uq;
                }
            }
}

static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; i++) f *= i; return f; }

/* Symmetric derivative values D[a][b][c] = d^(a,b,c) (1/|R|), a+b+c <= nmax. */
void orc_green_derivs(const double R[3], int nmax, double *out /* JD^3 */)
{
    double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    double r = sqrt(r2);
    double ul[3] = {2.0 * R[0] / r2, 2.0 * R[1] / r2, 2.0 * R[2] / r2};
    double uq = 1.0 / r2;
    jet_t pw, tmp, acc;
    jet_zero(pw); jet_zero(acc);
    pw[0][0][0] = 1.0;
    double binom = 1.0;   /* binomial(-1/2, k) */
    for (int k = 0; k <= nmax; k++) {
        for (int i = 0; i <= nmax; i++)
            for (int j = 0; i + j <= nmax; j++)
                for (int l = 0; i + j + l <= nmax; l++)
                    acc[i][j][l] += binom * pw[i][j][l];
        jet_mul_u(tmp, pw, ul, uq, nmax);
        memcpy(pw, tmp, sizeof(jet_t));
        binom *= (-0.5 - (double)k) / (double)(k + 1);
    }
    for (int i = 0; i < JD; i++)
        for (int j = 0; j < JD; j++)
            for (int l = 0; l < JD; l++) {
                double v = 0.0;
                if (i + j + l <= nmax) v = acc[i][j][l] / r * fact(i) * fact(j) * fact(l);
                out[(i * JD + j) * JD + l] = v;
            }
}

/* Full 3^n tensor of the n-th derivative from the symmetric values. */
static void full_from_sym(const double *sym, int n, double *full)
{
    int sz = ipow3(n);
    for (int idx = 0; idx < sz; idx++) {
        int cnt[3] = {0, 0, 0}, v = idx;
        for (int k = 0; k < n; k++) { cnt[v % 3]++; v /= 3; }
        full[idx] = sym[(cnt[0] * JD + cnt[1]) * JD + cnt[2]];
    }
}

void orc_green_deriv_full(const double R[3], int n, double *full)
{
    double sym[JD * JD * JD];
    orc_green_derivs(R, n, sym);
    full_from_sym(sym, n, full);
}

/* n-fold outer power d^(n) (Eq. 19 applied repeatedly). */
static void outer_power(const double d[3], int n, double *out)
{
    out[0] = 1.0;
    int sz = 1;
    for (int k = 1; k <= n; k++) {
        for (int idx = sz - 1; idx >= 0; idx--) {
            double v = out[idx];
            out[3 * idx + 0] = v * d[0];
            out[3 * idx + 1] = v * d[1];
            out[3 * idx + 2] = v * d[2];
        }
        sz *= 3;
    }
}

/* (T1^(n) (.) T2^(n-k)) accumulated with weight w into out^(k) (Eq. 18). */
static void inner_acc(const double *T1, int n, const double *T2, int k, double w,
                      double *out)
{
    int nk = n - k, szI = ipow3(k), szJ = ipow3(nk);
    for (int I = 0; I < szI; I++) {
        double s = 0.0;
        const double *row = T1 + (int64_t)I * szJ;
        for (int J = 0; J < szJ; J++) s += row[J] * T2[J];
        out[I] += w * s;
    }
}

/* ------------------------------------------------------------------------- */
/* Gravity: climb, walk, descent on the flat tree.                             */
/* ------------------------------------------------------------------------- */
typedef struct orc_grav {
    const orc_tree *t;
    int p, theta_mode;
    double G, theta_min;
    int64_t n, nc;
    double *xs, *ys, *zs, *mu;       /* tree order */
    double *s;                       /* COM, 3 per cell */
    double *mass, *rmax, *rcrit, *theta;
    double **M;                      /* M[c][off(n)] full multipoles n=0,2..p-1 */
    double **C;                      /* C[c][off(m)] full interaction tensors m=1..p */
    int moff[ORC_MAXP + 1], coff[ORC_MAXP + 2], msz, csz;
    double *ax, *ay, *az;            /* tree order accelerations */
    /* interaction records */
    int32_t *m2l; int64_t nm2l, cm2l;
    int32_t *p2p; int64_t np2p, cp2p;
    int64_t p2p_pairs;               /* moonlet pairs treated brute-force */
    int ncs, ncc_pre, ncc_post;
} orc_grav;

static void rec_push(int32_t **arr, int64_t *n, int64_t *cap, int32_t a, int32_t b)
{
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 1024;
        *arr = (int32_t *)realloc(*arr, (size_t)*cap * 2 * sizeof(int32_t));
    }
    (*arr)[2 * *n] = a; (*arr)[2 * *n + 1] = b;
    (*n)++;
}

orc_grav *orc_grav_new(const orc_tree *t, const double *x, const double *y,
                       const double *z, const double *m, double G, int p,
                       double theta_min, int theta_mode)
{
    orc_grav *g = (orc_grav *)calloc(1, sizeof(orc_grav));
    g->t = t; g->p = p; g->G = G; g->theta_min = theta_min; g->theta_mode = theta_mode;
    int64_t n = t->n, nc = t->ncells;
    g->n = n; g->nc = nc;
    g->xs = (double *)malloc((size_t)n * 8); g->ys = (double *)malloc((size_t)n * 8);
    g->zs = (double *)malloc((size_t)n * 8); g->mu = (double *)malloc((size_t)n * 8);
    for (int64_t k = 0; k < n; k++) {
        int64_t i = t->perm[k];
        g->xs[k] = x[i]; g->ys[k] = y[i]; g->zs[k] = z[i]; g->mu[k] = G * m[i];
    }
    g->s = (double *)malloc((size_t)nc * 3 * 8);
    g->mass = (double *)malloc((size_t)nc * 8);
    g->rmax = (double *)malloc((size_t)nc * 8);
    g->rcrit = (double *)malloc((size_t)nc * 8);
    g->theta = (double *)malloc((size_t)nc * 8);
    /* layout of the multipole and interaction tensor blocks per cell */
    int off = 0;
    for (int k = 0; k <= ORC_MAXP; k++) {
        g->moff[k] = -1;
        if (k < p && k != 1) { g->moff[k] = off; off += ipow3(k); }
    }
    g->msz = off;
    off = 0;
    for (int k = 0; k <= ORC_MAXP + 1; k++) {
        g->coff[k] = -1;
        if (k >= 1 && k <= p) { g->coff[k] = off; off += ipow3(k); }
    }
    g->csz = off;
    g->M = (double **)calloc((size_t)nc, sizeof(double *));
    g->C = (double **)calloc((size_t)nc, sizeof(double *));
    for (int64_t c = 0; c < nc; c++) {
        g->M[c] = (double *)calloc((size_t)(g->msz > 0 ? g->msz : 1), 8);
        g->C[c] = (double *)calloc((size_t)(g->csz > 0 ? g->csz : 1), 8);
    }
    g->ax = (double *)calloc((size_t)n, 8);
    g->ay = (double *)calloc((size_t)n, 8);
    g->az = (double *)calloc((size_t)n, 8);

    /* climb, children before parents: reverse breadth-first order */
    for (int64_t c = nc - 1; c >= 0; c--) {
        double sc[3];
        if (t->nchild[c] == 0) {
            /* leaf: moonlets are the children (Eqs. 10-11 with r_max,a = 0) */
            double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            for (int64_t k = t->first[c]; k < t->first[c] + t->count[c]; k++) {
                M += g->mu[k];
                sx += g->mu[k] * g->xs[k];
                sy += g->mu[k] * g->ys[k];
                sz += g->mu[k] * g->zs[k];
            }
            sc[0] = sx / M; sc[1] = sy / M; sc[2] = sz / M;
            double rm = 0.0;
            for (int64_t k = t->first[c]; k < t->first[c] + t->count[c]; k++) {
                double pk[3] = {g->xs[k], g->ys[k], g->zs[k]};
                double d = 0.0 + dist3(pk, sc);
                if (d > rm) rm = d;
            }
            g->mass[c] = M;
            g->rmax[c] = rm;
        } else {
            double M = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
            int64_t a0 = t->child_first[c], a1 = a0 + t->nchild[c];
            for (int64_t a = a0; a < a1; a++) M += g->mass[a];
            for (int64_t a = a0; a < a1; a++) {
                sx += g->mass[a] * g->s[3 * a];
                sy += g->mass[a] * g->s[3 * a + 1];
                sz += g->mass[a] * g->s[3 * a + 2];
            }
            sc[0] = sx / M; sc[1] = sy / M; sc[2] = sz / M;
            double rm = 0.0;
            for (int64_t a = a0; a < a1; a++) {
                double d = g->rmax[a] + dist3(&g->s[3 * a], sc);
                if (d > rm) rm = d;
            }
            g->mass[c] = M;
            g->rmax[c] = rm;
        }
        double fc = far_corner(t, c, sc);
        if (fc < g->rmax[c]) g->rmax[c] = fc;
        g->s[3 * c] = sc[0]; g->s[3 * c + 1] = sc[1]; g->s[3 * c + 2] = sc[2];
        /* multipoles straight from Eq. (20) */
        double pw[729];
        for (int64_t k = t->first[c]; k < t->first[c] + t->count[c]; k++) {
            double d[3] = {g->xs[k] - sc[0], g->ys[k] - sc[1], g->zs[k] - sc[2]};
            for (int nn = 0; nn < p; nn++) {
                if (g->moff[nn] < 0) continue;
                outer_power(d, nn, pw);
                double *Mn = g->M[c] + g->moff[nn];
                int sz = ipow3(nn);
                for (int J = 0; J < sz; J++) Mn[J] += g->mu[k] * pw[J];
            }
        }
    }
    double Mroot = g->mass[0];
    for (int64_t c = 0; c < nc; c++) {
        double th = theta_mode == 1 ? theta_min : orc_theta_of_mass(g->mass[c], Mroot, theta_min);
        g->theta[c] = th;
        g->rcrit[c] = g->rmax[c] / th;              /* Eq. (12) */
    }
    return g;
}

/* brute-force interaction of moonlets of A with moonlets of B (A != B) */
static void grav_p2p_pair(orc_grav *g, int64_t A, int64_t B)
{
    const orc_tree *t = g->t;
    for (int64_t i = t->first[A]; i < t->first[A] + t->count[A]; i++)
        for (int64_t j = t->first[B]; j < t->first[B] + t->count[B]; j++) {
            double dx = g->xs[j] - g->xs[i], dy = g->ys[j] - g->ys[i], dz = g->zs[j] - g->zs[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2), r3 = r2 * r;
            g->ax[i] += g->mu[j] * dx / r3; g->ay[i] += g->mu[j] * dy / r3;
            g->az[i] += g->mu[j] * dz / r3;
            g->ax[j] -= g->mu[i] * dx / r3; g->ay[j] -= g->mu[i] * dy / r3;
            g->az[j] -= g->mu[i] * dz / r3;
            g->p2p_pairs++;
        }
}

static void grav_p2p_self(orc_grav *g, int64_t A)
{
    const orc_tree *t = g->t;
    int64_t f = t->first[A], e = f + t->count[A];
    for (int64_t i = f; i < e; i++)
        for (int64_t j = i + 1; j < e; j++) {
            double dx = g->xs[j] - g->xs[i], dy = g->ys[j] - g->ys[i], dz = g->zs[j] - g->zs[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2), r3 = r2 * r;
            g->ax[i] += g->mu[j] * dx / r3; g->ay[i] += g->mu[j] * dy / r3;
            g->az[i] += g->mu[j] * dz / r3;
            g->ax[j] -= g->mu[i] * dx / r3; g->ay[j] -= g->mu[i] * dy / r3;
            g->az[j] -= g->mu[i] * dz / r3;
            g->p2p_pairs++;
        }
}

/* C^(m)_target += sum_{n=0, n!=1}^{p-m} (-1)^n/n! grad^(n+m) g(R) (.) M^(n)_source,
 * R = s_target - s_source (Eq. 25). */
static void m2l_one(orc_grav *g, int64_t tgt, int64_t src)
{
    int p = g->p;
    double R[3] = {g->s[3 * tgt] - g->s[3 * src], g->s[3 * tgt + 1] - g->s[3 * src + 1],
                   g->s[3 * tgt + 2] - g->s[3 * src + 2]};
    double sym[JD * JD * JD];
    orc_green_derivs(R, p, sym);
    static double Dfull[ORC_MAXP + 1][729];
    for (int k = 1; k <= p; k++) full_from_sym(sym, k, Dfull[k]);
    for (int m = 1; m <= p; m++) {
        double *Cm = g->C[tgt] + g->coff[m];
        for (int nn = 0; nn <= p - m; nn++) {
            if (nn == 1) continue;           /* M^(1) = 0 at the centre of mass */
            double w = ((nn & 1) ? -1.0 : 1.0) / fact(nn);
            inner_acc(Dfull[nn + m], nn + m, g->M[src] + g->moff[nn], m, w, Cm);
        }
    }
}

static int is_leaf(const orc_tree *t, int64_t c) { return t->nchild[c] == 0; }

static void grav_walk(orc_grav *g, int64_t A, int64_t B)
{
    const orc_tree *t = g->t;
    int64_t Na = t->count[A], Nb = t->count[B];
    if (A == B) {
        if (Na <= g->ncs || is_leaf(t, A)) {
            rec_push(&g->p2p, &g->np2p, &g->cp2p, (int32_t)A, (int32_t)A);
            grav_p2p_self(g, A);
        } else {
            int64_t c0 = t->child_first[A], c1 = c0 + t->nchild[A];
            for (int64_t a = c0; a < c1; a++)
                for (int64_t b = a; b < c1; b++) grav_walk(g, a, b);
        }
        return;
    }
    if (Na * Nb < (int64_t)g->ncc_pre) {
        rec_push(&g->p2p, &g->np2p, &g->cp2p, (int32_t)A, (int32_t)B);
        grav_p2p_pair(g, A, B);
    } else if (g->rcrit[A] + g->rcrit[B] <= dist3(&g->s[3 * A], &g->s[3 * B])) {
        rec_push(&g->m2l, &g->nm2l, &g->cm2l, (int32_t)A, (int32_t)B);
        m2l_one(g, A, B);
        m2l_one(g, B, A);
    } else if (Na * Nb < (int64_t)g->ncc_post || (is_leaf(t, A) && is_leaf(t, B))) {
        rec_push(&g->p2p, &g->np2p, &g->cp2p, (int32_t)A, (int32_t)B);
        grav_p2p_pair(g, A, B);
    } else if (is_leaf(t, B) || (!is_leaf(t, A) && g->rcrit[A] > g->rcrit[B])) {
        int64_t c0 = t->child_first[A], c1 = c0 + t->nchild[A];
        for (int64_t a = c0; a < c1; a++) grav_walk(g, a, B);
    } else {
        int64_t c0 = t->child_first[B], c1 = c0 + t->nchild[B];
        for (int64_t b = c0; b < c1; b++) grav_walk(g, A, b);
    }
}

/* Runs TreeWalk(root, root) then the descent; accelerations returned in input
 * order.  p = 0 means no mutual gravity at all. */
void orc_grav_run(orc_grav *g, int ncs, int ncc_pre, int ncc_post)
{
    const orc_tree *t = g->t;
    g->ncs = ncs; g->ncc_pre = ncc_pre; g->ncc_post = ncc_post;
    if (g->p == 0) return;
    grav_walk(g, 0, 0);
    /* descent, parents before children (Eq. 26) */
    int p = g->p;
    double pw[729];
    for (int64_t c = 0; c < g->nc; c++) {
        if (is_leaf(t, c)) continue;
        for (int64_t ch = t->child_first[c]; ch < t->child_first[c] + t->nchild[c]; ch++) {
            double d[3] = {g->s[3 * ch] - g->s[3 * c], g->s[3 * ch + 1] - g->s[3 * c + 1],
                           g->s[3 * ch + 2] - g->s[3 * c + 2]};
            for (int m = 1; m <= p; m++) {
                double *Cm = g->C[ch] + g->coff[m];
                for (int nn = 0; nn <= p - m; nn++) {
                    outer_power(d, nn, pw);
                    inner_acc(g->C[c] + g->coff[m + nn], m + nn, pw, m, 1.0 / fact(nn), Cm);
                }
            }
        }
    }
    /* evaluation at the moonlets of every leaf: C^(1)(x_i) by Eq. (26) */
    for (int64_t c = 0; c < g->nc; c++) {
        if (!is_leaf(t, c)) continue;
        for (int64_t k = t->first[c]; k < t->first[c] + t->count[c]; k++) {
            double d[3] = {g->xs[k] - g->s[3 * c], g->ys[k] - g->s[3 * c + 1],
                           g->zs[k] - g->s[3 * c + 2]};
            double acc[3] = {0.0, 0.0, 0.0};
            for (int nn = 0; nn <= p - 1; nn++) {
                outer_power(d, nn, pw);
                inner_acc(g->C[c] + g->coff[1 + nn], 1 + nn, pw, 1, 1.0 / fact(nn), acc);
            }
            g->ax[k] += acc[0]; g->ay[k] += acc[1]; g->az[k] += acc[2];
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Standard tree code (Alg. 1, Sect. 3.4.4): every moonlet walks the tree from  */
/* the root on its own.  A cell B with fewer than N_cb,pre moonlets is summed   */
/* directly; a cell well separated from the moonlet (|x - s_B| >= r_crit,B, and */
/* x != s_B: a cell whose moonlets all sit at x, r_crit = 0, is not separated   */
/* from a moonlet there, where C^(1) would be singular)                          */
/* contributes C^(1)(x) = sum_{n=0, n!=1}^{p-1} (-1)^n/n! grad^(n+1) g(R) (.)   */
/* M^(n)_B with R = x - s_B; a leaf or a cell with fewer than N_cb,post moonlets */
/* is summed directly; otherwise the walk goes on into B's children.            */
/* ------------------------------------------------------------------------- */
static void std_walk(orc_grav *g, int64_t k, int64_t B, int ncb_pre, int ncb_post, double *acc)
{
    const orc_tree *t = g->t;
    const int64_t Nb = t->count[B];
    const double x[3] = {g->xs[k], g->ys[k], g->zs[k]};
    int direct = 0;
    if (Nb < (int64_t)ncb_pre) {
        direct = 1;
    } else if (dist3(x, &g->s[3 * B]) >= g->rcrit[B] && dist3(x, &g->s[3 * B]) > 0.0) {
        int p = g->p;
        double R[3] = {x[0] - g->s[3 * B], x[1] - g->s[3 * B + 1], x[2] - g->s[3 * B + 2]};
        double sym[JD * JD * JD];
        orc_green_derivs(R, p, sym);
        static double Dfull[ORC_MAXP + 1][729];
        for (int q = 1; q <= p; q++) full_from_sym(sym, q, Dfull[q]);
        for (int nn = 0; nn <= p - 1; nn++) {
            if (nn == 1) continue;
            double w = ((nn & 1) ? -1.0 : 1.0) / fact(nn);
            inner_acc(Dfull[nn + 1], nn + 1, g->M[B] + g->moff[nn], 1, w, acc);
        }
        return;
    } else if (Nb < (int64_t)ncb_post || is_leaf(t, B)) {
        direct = 1;
    }
    if (direct) {
        for (int64_t j = t->first[B]; j < t->first[B] + Nb; j++) {
            double dx = g->xs[j] - x[0], dy = g->ys[j] - x[1], dz = g->zs[j] - x[2];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2), r3 = r2 * r;
            acc[0] += g->mu[j] * dx / r3;
            acc[1] += g->mu[j] * dy / r3;
            acc[2] += g->mu[j] * dz / r3;
        }
        return;
    }
    for (int64_t b = t->child_first[B]; b < t->child_first[B] + t->nchild[B]; b++)
        std_walk(g, k, b, ncb_pre, ncb_post, acc);
}

/* Accelerations by the standard tree code, replacing the falcON ones of g
 * (input order through orc_grav_accel).  p = 0: no mutual gravity. */
void orc_grav_run_std(orc_grav *g, int ncb_pre, int ncb_post)
{
    for (int64_t k = 0; k < g->n; k++) { g->ax[k] = 0.0; g->ay[k] = 0.0; g->az[k] = 0.0; }
    if (g->p == 0) return;
    for (int64_t k = 0; k < g->n; k++) {
        double acc[3] = {0.0, 0.0, 0.0};
        std_walk(g, k, 0, ncb_pre, ncb_post, acc);
        g->ax[k] = acc[0]; g->ay[k] = acc[1]; g->az[k] = acc[2];
    }
}

/* The standard tree's accelerations of a few moonlets only (input indices in     */
/* targets; out: nt x 3), for checks at sizes where walking every moonlet is slow. */
void orc_grav_run_std_targets(orc_grav *g, int ncb_pre, int ncb_post, const int64_t *targets,
                              int64_t nt, double *out)
{
    int64_t *where = (int64_t *)malloc((size_t)g->n * sizeof(int64_t));
    for (int64_t k = 0; k < g->n; k++) where[g->t->perm[k]] = k;
    for (int64_t q = 0; q < nt; q++) {
        double acc[3] = {0.0, 0.0, 0.0};
        if (g->p > 0) std_walk(g, where[targets[q]], 0, ncb_pre, ncb_post, acc);
        out[3 * q] = acc[0]; out[3 * q + 1] = acc[1]; out[3 * q + 2] = acc[2];
    }
    free(where);
}

void orc_grav_accel(const orc_grav *g, double *ax, double *ay, double *az)
{
    for (int64_t k = 0; k < g->n; k++) {
        int64_t i = g->t->perm[k];
        ax[i] = g->ax[k]; ay[i] = g->ay[k]; az[i] = g->az[k];
    }
}

void orc_grav_counts(const orc_grav *g, int64_t *out /* [3] */)
{
    out[0] = g->nm2l; out[1] = g->np2p; out[2] = g->p2p_pairs;
}

void orc_grav_lists(const orc_grav *g, int32_t *m2l, int32_t *p2p)
{
    if (g->nm2l) memcpy(m2l, g->m2l, (size_t)g->nm2l * 2 * sizeof(int32_t));
    if (g->np2p) memcpy(p2p, g->p2p, (size_t)g->np2p * 2 * sizeof(int32_t));
}

void orc_grav_cells(const orc_grav *g, double *s, double *mass, double *rmax,
                    double *rcrit)
{
    memcpy(s, g->s, (size_t)g->nc * 3 * 8);
    memcpy(mass, g->mass, (size_t)g->nc * 8);
    memcpy(rmax, g->rmax, (size_t)g->nc * 8);
    memcpy(rcrit, g->rcrit, (size_t)g->nc * 8);
}

int orc_grav_msize(const orc_grav *g) { return g->msz; }
int orc_grav_csize(const orc_grav *g) { return g->csz; }

/* full multipole / interaction tensors of one cell, blocks in increasing order */
void orc_grav_cell_tensors(const orc_grav *g, int64_t c, double *M, double *C)
{
    if (g->msz) memcpy(M, g->M[c], (size_t)g->msz * 8);
    if (g->csz) memcpy(C, g->C[c], (size_t)g->csz * 8);
}

void orc_grav_free(orc_grav *g)
{
    if (!g) return;
    for (int64_t c = 0; c < g->nc; c++) { free(g->M[c]); free(g->C[c]); }
    free(g->M); free(g->C);
    free(g->xs); free(g->ys); free(g->zs); free(g->mu);
    free(g->s); free(g->mass); free(g->rmax); free(g->rcrit); free(g->theta);
    free(g->ax); free(g->ay); free(g->az);
    free(g->m2l); free(g->p2p);
    free(g);
}

/* Single-cell-pair expansion check: the acceleration at target points due to
 * source moonlets via P2M (Eq. 20) -> M2L (Eq. 25) at s_A -> shift (Eq. 26) to
 * each target.  Used to pin the expansion machinery against the exact field. */
void orc_expansion_field(const double *xs, const double *ys, const double *zs,
                         const double *mus, int64_t ns, const double sA[3],
                         const double *xt, const double *yt, const double *zt,
                         int64_t nt, int p, double *ax, double *ay, double *az)
{
    double M = 0.0, sB[3] = {0, 0, 0};
    for (int64_t k = 0; k < ns; k++) {
        M += mus[k]; sB[0] += mus[k] * xs[k]; sB[1] += mus[k] * ys[k]; sB[2] += mus[k] * zs[k];
    }
    sB[0] /= M; sB[1] /= M; sB[2] /= M;
    int moff[ORC_MAXP + 1], coff[ORC_MAXP + 2], off = 0;
    for (int k = 0; k <= ORC_MAXP; k++) { moff[k] = -1; if (k < p && k != 1) { moff[k] = off; off += ipow3(k); } }
    double *Mt = (double *)calloc((size_t)(off + 1), 8);
    off = 0;
    for (int k = 0; k <= ORC_MAXP + 1; k++) { coff[k] = -1; if (k >= 1 && k <= p) { coff[k] = off; off += ipow3(k); } }
    double *Ct = (double *)calloc((size_t)(off + 1), 8);
    double pw[729];
    for (int64_t k = 0; k < ns; k++) {
        double d[3] = {xs[k] - sB[0], ys[k] - sB[1], zs[k] - sB[2]};
        for (int nn = 0; nn < p; nn++) {
            if (moff[nn] < 0) continue;
            outer_power(d, nn, pw);
            for (int J = 0; J < ipow3(nn); J++) Mt[moff[nn] + J] += mus[k] * pw[J];
        }
    }
    double R[3] = {sA[0] - sB[0], sA[1] - sB[1], sA[2] - sB[2]};
    double sym[JD * JD * JD];
    orc_green_derivs(R, p, sym);
    static double Dfull[ORC_MAXP + 1][729];
    for (int k = 1; k <= p; k++) full_from_sym(sym, k, Dfull[k]);
    for (int m = 1; m <= p; m++)
        for (int nn = 0; nn <= p - m; nn++) {
            if (nn == 1) continue;
            double w = ((nn & 1) ? -1.0 : 1.0) / fact(nn);
            inner_acc(Dfull[nn + m], nn + m, Mt + moff[nn], m, w, Ct + coff[m]);
        }
    for (int64_t i = 0; i < nt; i++) {
        double d[3] = {xt[i] - sA[0], yt[i] - sA[1], zt[i] - sA[2]};
        double acc[3] = {0, 0, 0};
        for (int nn = 0; nn <= p - 1; nn++) {
            outer_power(d, nn, pw);
            inner_acc(Ct + coff[1 + nn], 1 + nn, pw, 1, 1.0 / fact(nn), acc);
        }
        ax[i] = acc[0]; ay[i] = acc[1]; az[i] = acc[2];
    }
    free(Mt); free(Ct);
}

/* Shift of interaction tensors (Eq. 26) on full tensors, exported for the
 * polynomial re-expansion pin.  Cin/Cout hold blocks m = 1..p. */
void orc_shift_C(const double *Cin, int p, const double d[3], double *Cout)
{
    int coff[ORC_MAXP + 2], off = 0;
    for (int k = 0; k <= ORC_MAXP + 1; k++) { coff[k] = -1; if (k >= 1 && k <= p) { coff[k] = off; off += ipow3(k); } }
    memset(Cout, 0, (size_t)off * 8);
    double pw[729];
    for (int m = 1; m <= p; m++)
        for (int nn = 0; nn <= p - m; nn++) {
            outer_power(d, nn, pw);
            inner_acc(Cin + coff[m + nn], m + nn, pw, m, 1.0 / fact(nn), Cout + coff[m]);
        }
}

/* ------------------------------------------------------------------------- */
/* Collision search with the same tree (Eqs. 7-9, Alg. 2 in italic form).     */
/* ------------------------------------------------------------------------- */
typedef struct orc_coll {
    const orc_tree *t;
    int64_t n, nc;
    double *xs, *ys, *zs, *vxs, *vys, *vzs, *Rs;
    double *sbar, *rmax, *rcrit;
    double dt;
    int ncs, ncc_pre, ncc_post;
    int64_t *pairs, npairs, cpairs;
    int32_t *cand; int64_t ncand, ccand;
    int64_t tests;
} orc_coll;

orc_coll *orc_coll_new(const orc_tree *t, const double *x, const double *y,
                       const double *z, const double *vx, const double *vy,
                       const double *vz, const double *R, double dt)
{
    orc_coll *c = (orc_coll *)calloc(1, sizeof(orc_coll));
    int64_t n = t->n, nc = t->ncells;
    c->t = t; c->n = n; c->nc = nc; c->dt = dt;
    double **arrs[7] = {&c->xs, &c->ys, &c->zs, &c->vxs, &c->vys, &c->vzs, &c->Rs};
    const double *src[7] = {x, y, z, vx, vy, vz, R};
    for (int a = 0; a < 7; a++) {
        *arrs[a] = (double *)malloc((size_t)n * 8);
        for (int64_t k = 0; k < n; k++) (*arrs[a])[k] = src[a][t->perm[k]];
    }
    c->sbar = (double *)malloc((size_t)nc * 3 * 8);
    c->rmax = (double *)malloc((size_t)nc * 8);
    c->rcrit = (double *)malloc((size_t)nc * 8);
    for (int64_t A = nc - 1; A >= 0; A--) {
        double sc[3], rm = 0.0, ex = 0.0;
        int64_t NA = t->count[A];
        if (t->nchild[A] == 0) {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            for (int64_t k = t->first[A]; k < t->first[A] + NA; k++) {
                sx += c->xs[k]; sy += c->ys[k]; sz += c->zs[k];
            }
            sc[0] = sx / (double)NA; sc[1] = sy / (double)NA; sc[2] = sz / (double)NA;
            for (int64_t k = t->first[A]; k < t->first[A] + NA; k++) {
                double pk[3] = {c->xs[k], c->ys[k], c->zs[k]};
                double d = 0.0 + dist3(pk, sc);
                if (d > rm) rm = d;
                double v = sqrt(c->vxs[k] * c->vxs[k] + c->vys[k] * c->vys[k] +
                                c->vzs[k] * c->vzs[k]);
                double e = (c->Rs[k] + dt * v) - 0.0;     /* r_crit,a - r_max,a */
                if (e > ex) ex = e;
            }
        } else {
            double sx = 0.0, sy = 0.0, sz = 0.0;
            int64_t a0 = t->child_first[A], a1 = a0 + t->nchild[A];
            for (int64_t a = a0; a < a1; a++) {
                double na = (double)t->count[a];
                sx += na * c->sbar[3 * a]; sy += na * c->sbar[3 * a + 1];
                sz += na * c->sbar[3 * a + 2];
            }
            sc[0] = sx / (double)NA; sc[1] = sy / (double)NA; sc[2] = sz / (double)NA;
            for (int64_t a = a0; a < a1; a++) {
                double d = c->rmax[a] + dist3(&c->sbar[3 * a], sc);
                if (d > rm) rm = d;
                double e = c->rcrit[a] - c->rmax[a];
                if (e > ex) ex = e;
            }
        }
        double fc = far_corner(t, A, sc);
        if (fc < rm) rm = fc;
        c->sbar[3 * A] = sc[0]; c->sbar[3 * A + 1] = sc[1]; c->sbar[3 * A + 2] = sc[2];
        c->rmax[A] = rm;
        c->rcrit[A] = rm + ex;                           /* Eq. (9) */
    }
    return c;
}

static void coll_record(orc_coll *c, int64_t a, int64_t b)
{
    int64_t i = c->t->perm[a], j = c->t->perm[b];
    if (i > j) { int64_t t = i; i = j; j = t; }
    if (c->npairs == c->cpairs) {
        c->cpairs = c->cpairs ? 2 * c->cpairs : 256;
        c->pairs = (int64_t *)realloc(c->pairs, (size_t)c->cpairs * 2 * 8);
    }
    c->pairs[2 * c->npairs] = i; c->pairs[2 * c->npairs + 1] = j;
    c->npairs++;
}

static void coll_test(orc_coll *c, int64_t a, int64_t b)
{
    c->tests++;
    if (orc_pair_test(c->xs[a], c->ys[a], c->zs[a], c->vxs[a], c->vys[a], c->vzs[a], c->Rs[a],
                      c->xs[b], c->ys[b], c->zs[b], c->vxs[b], c->vys[b], c->vzs[b], c->Rs[b],
                      c->dt))
        coll_record(c, a, b);
}

static void coll_brute_self(orc_coll *c, int64_t A)
{
    int64_t f = c->t->first[A], e = f + c->t->count[A];
    rec_push(&c->cand, &c->ncand, &c->ccand, (int32_t)A, (int32_t)A);
    for (int64_t a = f; a < e; a++)
        for (int64_t b = a + 1; b < e; b++) coll_test(c, a, b);
}

static void coll_brute_pair(orc_coll *c, int64_t A, int64_t B)
{
    const orc_tree *t = c->t;
    rec_push(&c->cand, &c->ncand, &c->ccand, (int32_t)A, (int32_t)B);
    for (int64_t a = t->first[A]; a < t->first[A] + t->count[A]; a++)
        for (int64_t b = t->first[B]; b < t->first[B] + t->count[B]; b++) coll_test(c, a, b);
}

static void coll_walk(orc_coll *c, int64_t A, int64_t B)
{
    const orc_tree *t = c->t;
    int64_t Na = t->count[A], Nb = t->count[B];
    if (A == B) {
        if (Na <= c->ncs || is_leaf(t, A)) coll_brute_self(c, A);
        else {
            int64_t c0 = t->child_first[A], c1 = c0 + t->nchild[A];
            for (int64_t a = c0; a < c1; a++)
                for (int64_t b = a; b < c1; b++) coll_walk(c, a, b);
        }
        return;
    }
    if (Na * Nb < (int64_t)c->ncc_pre) coll_brute_pair(c, A, B);
    else if (c->rcrit[A] + c->rcrit[B] <= dist3(&c->sbar[3 * A], &c->sbar[3 * B])) {
        /* well separated: no collision possible */
    } else if (Na * Nb < (int64_t)c->ncc_post || (is_leaf(t, A) && is_leaf(t, B)))
        coll_brute_pair(c, A, B);
    else if (is_leaf(t, B) || (!is_leaf(t, A) && c->rcrit[A] > c->rcrit[B])) {
        int64_t c0 = t->child_first[A], c1 = c0 + t->nchild[A];
        for (int64_t a = c0; a < c1; a++) coll_walk(c, a, B);
    } else {
        int64_t c0 = t->child_first[B], c1 = c0 + t->nchild[B];
        for (int64_t b = c0; b < c1; b++) coll_walk(c, A, b);
    }
}

static int cmp_pair(const void *a, const void *b)
{
    const int64_t *p = (const int64_t *)a, *q = (const int64_t *)b;
    if (p[0] != q[0]) return p[0] < q[0] ? -1 : 1;
    if (p[1] != q[1]) return p[1] < q[1] ? -1 : 1;
    return 0;
}

int64_t orc_coll_run(orc_coll *c, int ncs, int ncc_pre, int ncc_post)
{
    c->ncs = ncs; c->ncc_pre = ncc_pre; c->ncc_post = ncc_post;
    coll_walk(c, 0, 0);
    if (c->npairs) qsort(c->pairs, (size_t)c->npairs, 2 * sizeof(int64_t), cmp_pair);
    return c->npairs;
}

void orc_coll_pairs(const orc_coll *c, int64_t *out)
{
    if (c->npairs) memcpy(out, c->pairs, (size_t)c->npairs * 2 * 8);
}

int64_t orc_coll_ncand(const orc_coll *c) { return c->ncand; }
int64_t orc_coll_ntests(const orc_coll *c) { return c->tests; }
void orc_coll_cand(const orc_coll *c, int32_t *out)
{
    if (c->ncand) memcpy(out, c->cand, (size_t)c->ncand * 2 * sizeof(int32_t));
}
void orc_coll_cells(const orc_coll *c, double *sbar, double *rmax, double *rcrit)
{
    memcpy(sbar, c->sbar, (size_t)c->nc * 3 * 8);
    memcpy(rmax, c->rmax, (size_t)c->nc * 8);
    memcpy(rcrit, c->rcrit, (size_t)c->nc * 8);
}

void orc_coll_free(orc_coll *c)
{
    if (!c) return;
    free(c->xs); free(c->ys); free(c->zs); free(c->vxs); free(c->vys); free(c->vzs);
    free(c->Rs); free(c->sbar); free(c->rmax); free(c->rcrit); free(c->pairs);
    free(c->cand);
    free(c);
}

/* ------------------------------------------------------------------------- */
/* Plain definitions: direct sum and brute-force pair scan.                    */
/* ------------------------------------------------------------------------- */
static void neumaier_add(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v)) *c += (*s - t) + v;
    else *c += (v - t) + *s;
    *s = t;
}

/* a_i = sum_{j != i} G m_j (x_j - x_i)/|x_j - x_i|^3 for the listed targets. */
void orc_direct_sum(const double *x, const double *y, const double *z, const double *m,
                    int64_t n, double G, const int64_t *targets, int64_t nt, double *ax,
                    double *ay, double *az)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t k = 0; k < nt; k++) {
        int64_t i = targets[k];
        double sx = 0, cx = 0, sy = 0, cy = 0, sz = 0, cz = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2);
            double f = G * m[j] / (r2 * r);
            neumaier_add(&sx, &cx, f * dx);
            neumaier_add(&sy, &cy, f * dy);
            neumaier_add(&sz, &cz, f * dz);
        }
        ax[k] = sx + cx; ay[k] = sy + cy; az[k] = sz + cz;
    }
}

/* All colliding pairs (i<j), sorted; returns the count (may exceed cap, in which
 * case only the first cap found are stored, unsorted beyond that point). */
int64_t orc_pairs_brute(const double *x, const double *y, const double *z,
                        const double *vx, const double *vy, const double *vz,
                        const double *R, int64_t n, double dt, int64_t *out, int64_t cap)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
        for (int64_t j = i + 1; j < n; j++) {
            if (orc_pair_test(x[i], y[i], z[i], vx[i], vy[i], vz[i], R[i],
                              x[j], y[j], z[j], vx[j], vy[j], vz[j], R[j], dt)) {
                int64_t slot;
#pragma omp atomic capture
                slot = total++;
                if (slot < cap) { out[2 * slot] = i; out[2 * slot + 1] = j; }
            }
        }
    }
    if (total <= cap) qsort(out, (size_t)total, 2 * sizeof(int64_t), cmp_pair);
    return total;
}

/* Partners j of each listed moonlet i with a collision in the next dt; writes
 * sorted pairs (min, max).  Used to check huge inputs one moonlet at a time. */
int64_t orc_pairs_of(const double *x, const double *y, const double *z, const double *vx,
                     const double *vy, const double *vz, const double *R, int64_t n,
                     double dt, const int64_t *targets, int64_t nt, int64_t *out, int64_t cap)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nt; k++) {
        int64_t i = targets[k];
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            if (orc_pair_test(x[i], y[i], z[i], vx[i], vy[i], vz[i], R[i],
                              x[j], y[j], z[j], vx[j], vy[j], vz[j], R[j], dt)) {
                int64_t slot;
#pragma omp atomic capture
                slot = total++;
                if (slot < cap) {
                    out[2 * slot] = i < j ? i : j;
                    out[2 * slot + 1] = i < j ? j : i;
                }
            }
        }
    }
    if (total <= cap) qsort(out, (size_t)total, 2 * sizeof(int64_t), cmp_pair);
    return total;
}

/* ------------------------------------------------------------------------- */
/* Every colliding pair (i < j) of Sect. 3.1, Eqs. (1)-(2), for inputs too     */
/* large for the all-pairs scan.  A pair that touches at a time t in [0, dt]    */
/* was at most R_i + R_j + t |v_i - v_j| <= reach_i + reach_j apart at t = 0,   */
/* reach = R + dt |v|.  With cubic cells of side h > 2 max(reach) (a relative  */
/* margin of 1e-6 absorbs rounding in the cell coordinates), such a pair sits   */
/* in the same or adjacent cells, so testing every pair of those cells with    */
/* orc_pair_test -- the same call, same argument order (i first) as the        */
/* all-pairs scan -- gives exactly the all-pairs set.  Nothing of the tree is   */
/* used.  Returns the count; pairs sorted as orc_pairs_brute.                  */
/* ------------------------------------------------------------------------- */
typedef struct { int64_t c[3]; int64_t id; } grid_ent;

static int cmp_grid_cell(const int64_t *a, const int64_t *b)
{
    for (int k = 0; k < 3; k++)
        if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
    return 0;
}

static int cmp_grid_ent(const void *a, const void *b)
{
    const grid_ent *p = (const grid_ent *)a, *q = (const grid_ent *)b;
    int r = cmp_grid_cell(p->c, q->c);
    if (r) return r;
    return p->id < q->id ? -1 : (p->id > q->id);
}

/* first entry whose cell is not below `cell` */
static int64_t grid_lower(const grid_ent *e, int64_t n, const int64_t cell[3])
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (cmp_grid_cell(e[mid].c, cell) < 0) lo = mid + 1; else hi = mid;
    }
    return lo;
}

int64_t orc_pairs_grid(const double *x, const double *y, const double *z, const double *vx,
                       const double *vy, const double *vz, const double *R, int64_t n,
                       double dt, int64_t *out, int64_t cap)
{
    double reach = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double r = R[i] + dt * sqrt(vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]);
        if (r > reach) reach = r;
    }
    if (!(reach > 0.0) || n < 2) return 0;   /* no radius and no motion: no contact */
    double h = 2.0 * reach * (1.0 + 1e-6);
    grid_ent *e = (grid_ent *)malloc((size_t)n * sizeof(grid_ent));
    for (int64_t i = 0; i < n; i++) {
        e[i].c[0] = (int64_t)floor(x[i] / h);
        e[i].c[1] = (int64_t)floor(y[i] / h);
        e[i].c[2] = (int64_t)floor(z[i] / h);
        e[i].id = i;
    }
    qsort(e, (size_t)n, sizeof(grid_ent), cmp_grid_ent);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t k = 0; k < n; k++) {
        int64_t i = e[k].id;
        for (int d = 0; d < 27; d++) {
            int64_t cell[3] = {e[k].c[0] + d % 3 - 1, e[k].c[1] + (d / 3) % 3 - 1,
                               e[k].c[2] + d / 9 - 1};
            for (int64_t m = grid_lower(e, n, cell); m < n && !cmp_grid_cell(e[m].c, cell); m++) {
                int64_t j = e[m].id;
                if (j <= i) continue;
                if (orc_pair_test(x[i], y[i], z[i], vx[i], vy[i], vz[i], R[i],
                                  x[j], y[j], z[j], vx[j], vy[j], vz[j], R[j], dt)) {
                    int64_t slot;
#pragma omp atomic capture
                    slot = total++;
                    if (slot < cap) { out[2 * slot] = i; out[2 * slot + 1] = j; }
                }
            }
        }
    }
    free(e);
    if (total <= cap) qsort(out, (size_t)total, 2 * sizeof(int64_t), cmp_pair);
    return total;
}

/* ------------------------------------------------------------------------- */
/* Mesh module (Sect. 3.3).  A gamma-mesh of cubic cells of side gamma, cell    */
/* (floor(x/gamma), floor(y/gamma), floor(z/gamma)); the neighbourhood of a     */
/* moonlet is its own cell and the 26 adjacent ones.  Pairs of moonlets in each */
/* other's neighbourhood interact (gravity) and are tested for collision.       */
/* A moonlet with diameter 2R > gamma is kept out of the mesh and interacts     */
/* with every other moonlet; for gravity, so do the three most massive          */
/* moonlets.  Everything here is brute force over all pairs.                    */
/* ------------------------------------------------------------------------- */

#define ORC_PI 3.14159265358979323846

/* Eq. (4): the largest mesh size that leaves x moonlets on average in a        */
/* neighbourhood (27 cells) of a disk of aspect ratio h/r inside radius R_max. */
double orc_mesh_gamma_crit(double x, double N, double aspect, double R_max)
{
    double s = aspect * aspect / (1.0 + aspect * aspect);
    return pow(4.0 * ORC_PI * x / (81.0 * N), 1.0 / 3.0) * pow(s, 1.0 / 6.0) * R_max;
}

/* Eq. (5): the smallest aspect ratio for which moonlets of the mean radius of  */
/* N moonlets of total mass one Moon fit the critical mesh (2R <= gamma); the  */
/* argument is R_Moon / R_max.                                                  */
double orc_mesh_aspect_crit(double x, double moon_over_rmax)
{
    return 162.0 / (ORC_PI * x) * moon_over_rmax * moon_over_rmax * moon_over_rmax;
}

/* Eq. (6): the next mesh size from the measured mean neighbour count x'; no   */
/* smaller than gamma_min; with no neighbour at all (x' = 0) the mesh doubles. */
double orc_mesh_gamma_next(double gamma_prev, double x, double x_measured, double gamma_min)
{
    double g = x_measured > 0.0 ? gamma_prev * cbrt(x / x_measured) : 2.0 * gamma_prev;
    return g > gamma_min ? g : gamma_min;
}

static void mesh_cell(double x, double y, double z, double gamma, int64_t c[3])
{
    c[0] = (int64_t)floor(x / gamma);
    c[1] = (int64_t)floor(y / gamma);
    c[2] = (int64_t)floor(z / gamma);
}

static int mesh_adjacent(const int64_t a[3], const int64_t b[3])
{
    for (int k = 0; k < 3; k++)
        if (a[k] - b[k] > 1 || b[k] - a[k] > 1) return 0;
    return 1;
}

/* flags[i]: 1 = out of the mesh (2R > gamma), 2 = one of the three most massive */
/* moonlets (larger mass first, equal masses by smaller index), 3 = both.        */
void orc_mesh_flags(const double *m, const double *R, int64_t n, double gamma, int32_t *flags)
{
    int64_t top[3] = {-1, -1, -1};
    for (int64_t i = 0; i < n; i++) {
        flags[i] = 2.0 * R[i] > gamma ? 1 : 0;
        /* insert i into the running top three (strictly larger mass goes first) */
        for (int k = 0; k < 3; k++) {
            if (top[k] < 0 || m[i] > m[top[k]]) {
                for (int q = 2; q > k; q--) top[q] = top[q - 1];
                top[k] = i;
                break;
            }
        }
    }
    for (int k = 0; k < 3; k++)
        if (top[k] >= 0) flags[top[k]] |= 2;
}

/* mean over the moonlets in the mesh of the number of other moonlets of the   */
/* mesh in their neighbourhood (the x' of Eq. 6)                                */
double orc_mesh_neighbours(const double *x, const double *y, const double *z, const double *R,
                           int64_t n, double gamma)
{
    int64_t in = 0, pairs = 0;
    for (int64_t i = 0; i < n; i++) {
        if (2.0 * R[i] > gamma) continue;
        in++;
        int64_t ci[3];
        mesh_cell(x[i], y[i], z[i], gamma, ci);
        for (int64_t j = 0; j < n; j++) {
            if (j == i || 2.0 * R[j] > gamma) continue;
            int64_t cj[3];
            mesh_cell(x[j], y[j], z[j], gamma, cj);
            if (mesh_adjacent(ci, cj)) pairs++;
        }
    }
    return in > 0 ? (double)pairs / (double)in : 0.0;
}

/* does the pair (i, j) interact?  gravity: big = flags != 0; collisions:       */
/* big = out of the mesh only                                                    */
static int mesh_pair(const double *x, const double *y, const double *z, const int32_t *flags,
                     int big_mask, int64_t i, int64_t j, double gamma)
{
    if ((flags[i] & big_mask) || (flags[j] & big_mask)) return 1;
    if ((flags[i] & 1) || (flags[j] & 1)) return 0;
    int64_t ci[3], cj[3];
    mesh_cell(x[i], y[i], z[i], gamma, ci);
    mesh_cell(x[j], y[j], z[j], gamma, cj);
    return mesh_adjacent(ci, cj);
}

/* mutual accelerations over the interacting pairs (mu = G m) */
void orc_mesh_accel(const double *x, const double *y, const double *z, const double *m,
                    const double *R, int64_t n, double G, double gamma, double *ax, double *ay,
                    double *az)
{
    int32_t *flags = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    orc_mesh_flags(m, R, n, gamma, flags);
    for (int64_t i = 0; i < n; i++) {
        double a[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i || !mesh_pair(x, y, z, flags, 3, i, j, gamma)) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2), r3 = r2 * r, mu = G * m[j];
            a[0] += mu * dx / r3;
            a[1] += mu * dy / r3;
            a[2] += mu * dz / r3;
        }
        ax[i] = a[0]; ay[i] = a[1]; az[i] = a[2];
    }
    free(flags);
}

/* colliding pairs (i < j, increasing) among the pairs the mesh tests */
int64_t orc_mesh_pairs(const double *x, const double *y, const double *z, const double *vx,
                       const double *vy, const double *vz, const double *m, const double *R,
                       int64_t n, double gamma, double dt, int64_t *out, int64_t cap)
{
    int32_t *flags = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    orc_mesh_flags(m, R, n, gamma, flags);
    int64_t total = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = i + 1; j < n; j++) {
            if (!mesh_pair(x, y, z, flags, 1, i, j, gamma)) continue;
            if (!orc_pair_test(x[i], y[i], z[i], vx[i], vy[i], vz[i], R[i], x[j], y[j], z[j],
                               vx[j], vy[j], vz[j], R[j], dt))
                continue;
            if (total < cap) { out[2 * total] = i; out[2 * total + 1] = j; }
            total++;
        }
    free(flags);
    return total;
}

/* mesh accelerations of a few moonlets only (input indices; out: nt x 3) */
void orc_mesh_accel_targets(const double *x, const double *y, const double *z, const double *m,
                            const double *R, int64_t n, double G, double gamma,
                            const int64_t *targets, int64_t nt, double *out)
{
    int32_t *flags = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    orc_mesh_flags(m, R, n, gamma, flags);
    for (int64_t q = 0; q < nt; q++) {
        const int64_t i = targets[q];
        double a[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; j++) {
            if (j == i || !mesh_pair(x, y, z, flags, 3, i, j, gamma)) continue;
            double dx = x[j] - x[i], dy = y[j] - y[i], dz = z[j] - z[i];
            double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            double r = sqrt(r2), r3 = r2 * r, mu = G * m[j];
            a[0] += mu * dx / r3;
            a[1] += mu * dy / r3;
            a[2] += mu * dz / r3;
        }
        out[3 * q] = a[0]; out[3 * q + 1] = a[1]; out[3 * q + 2] = a[2];
    }
    free(flags);
}

/* colliding pairs of the mesh that involve one of the targets (i < j, increasing,
 * each once; targets sorted increasing and distinct) */
int64_t orc_mesh_pairs_of(const double *x, const double *y, const double *z, const double *vx,
                          const double *vy, const double *vz, const double *m, const double *R,
                          int64_t n, double gamma, double dt, const int64_t *targets, int64_t nt,
                          int64_t *out, int64_t cap)
{
    int32_t *flags = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    char *is_t = (char *)calloc((size_t)(n > 0 ? n : 1), 1);
    orc_mesh_flags(m, R, n, gamma, flags);
    for (int64_t q = 0; q < nt; q++) is_t[targets[q]] = 1;
    int64_t total = 0;
    for (int64_t q = 0; q < nt; q++) {
        const int64_t t = targets[q];
        for (int64_t j = 0; j < n; j++) {
            if (j == t) continue;
            if (is_t[j] && j < t) continue;           /* a pair of two targets once */
            if (!mesh_pair(x, y, z, flags, 1, t, j, gamma)) continue;
            if (!orc_pair_test(x[t], y[t], z[t], vx[t], vy[t], vz[t], R[t], x[j], y[j], z[j],
                               vx[j], vy[j], vz[j], R[j], dt))
                continue;
            if (total < cap) {
                out[2 * total] = t < j ? t : j;
                out[2 * total + 1] = t < j ? j : t;
            }
            total++;
        }
    }
    if (total <= cap) qsort(out, (size_t)total, 2 * sizeof(int64_t), cmp_pair);
    free(flags);
    free(is_t);
    return total;
}

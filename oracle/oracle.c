/*
 * FP64 CPU oracle for the tree/Hermite block-step force evaluation of
 * Fukushige & Kawai, "Hierarchical Tree Algorithm for Collisional N-body
 * Simulations on GRAPE" (PASJ; arXiv:1602.02832).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference against
 * which the GPU path is checked.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never calls
 * it and shares no code, header, table or helper with it.
 *
 * Everything is FP64, summed sequentially in the stated order; the file must
 * be compiled with -ffp-contract=off so every product and sum is rounded
 * exactly as written.  OpenMP is only used across independent particles or
 * groups, never inside one sum, so results do not depend on the thread count.
 *
 * Where the paper names an ingredient without a formula (the tree, the
 * groups, the opening test, the Hermite and Aarseth formulas) the reading
 * implemented here is the textbook one; each such reading is marked READING.
 *
 * Parity status per function (what pins it is in the test suite):
 *   hilbert keys, tree, node moments, groups, lists, predictor, list force,
 *   direct force, corrector, timestep, energy: pinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_BITS 21          /* bits per axis of the Peano-Hilbert key      */
#define ORC_MAX_LEVEL 21     /* deepest cell level                          */

/* ------------------------------------------------------------------------- */
/* Peano-Hilbert keys (Section 2: particles are rearranged in Peano-Hilbert   */
/* order so that interaction lists compress).  READING: the curve is the one  */
/* of J. Skilling, "Programming the Hilbert curve" (AIP Conf. Proc. 707,     */
/* 2004): the integer coordinates are converted to the "transposed" Hilbert   */
/* index, whose bits are then read most-significant first, x before y        */
/* before z in every triple.                                                  */
/* ------------------------------------------------------------------------- */
uint64_t orc_hilbert_key(uint32_t qx, uint32_t qy, uint32_t qz)
{
    uint32_t c[3] = {qx, qy, qz};
    const uint32_t top = 1u << (ORC_BITS - 1);
    /* undo the excess work of the recursive construction, from the top bit */
    for (uint32_t bit = top; bit > 1; bit >>= 1) {
        uint32_t low = bit - 1;
        for (int d = 0; d < 3; d++) {
            if (c[d] & bit) {
                c[0] ^= low;                          /* invert low bits of x */
            } else {
                uint32_t diff = (c[0] ^ c[d]) & low;  /* swap low bits x<->d  */
                c[0] ^= diff;
                c[d] ^= diff;
            }
        }
    }
    /* Gray encode */
    c[1] ^= c[0];
    c[2] ^= c[1];
    uint32_t flip = 0;
    for (uint32_t bit = top; bit > 1; bit >>= 1)
        if (c[2] & bit) flip ^= bit - 1;
    for (int d = 0; d < 3; d++) c[d] ^= flip;
    /* read the transposed index: bit b of x, then y, then z, from the top */
    uint64_t key = 0;
    for (int b = ORC_BITS - 1; b >= 0; b--)
        for (int d = 0; d < 3; d++)
            key = (key << 1) | (uint64_t)((c[d] >> b) & 1u);
    return key;
}

void orc_hilbert_keys(int64_t n, const uint32_t *q, uint64_t *out)
{
    for (int64_t i = 0; i < n; i++) out[i] = orc_hilbert_key(q[3 * i], q[3 * i + 1], q[3 * i + 2]);
}

/* ------------------------------------------------------------------------- */
/* Root cube and integer coordinates.  READING: lo = componentwise minimum,  */
/* side = 2^e with frexp(ext) = (f, e) for ext = the largest axis extent      */
/* (the smallest power of two strictly above ext), side = 1 if ext = 0.      */
/* q = floor((x - lo) * 2^21 / side), clamped to [0, 2^21 - 1].              */
/* ------------------------------------------------------------------------- */
void orc_root_box(int64_t n, const double *x, double lo[3], double *side)
{
    double hi[3];
    for (int d = 0; d < 3; d++) { lo[d] = x[d]; hi[d] = x[d]; }
    for (int64_t i = 1; i < n; i++)
        for (int d = 0; d < 3; d++) {
            double c = x[3 * i + d];
            if (c < lo[d]) lo[d] = c;
            if (c > hi[d]) hi[d] = c;
        }
    double ext = 0.0;
    for (int d = 0; d < 3; d++) {
        double e = hi[d] - lo[d];
        if (e > ext) ext = e;
    }
    if (ext == 0.0) { *side = 1.0; return; }
    int e2;
    frexp(ext, &e2);
    *side = ldexp(1.0, e2);
}

void orc_quantize(int64_t n, const double *x, const double lo[3], double side, uint32_t *q)
{
    const double scale = ldexp(1.0, ORC_BITS) / side;   /* exact power of two */
    const double qmax = ldexp(1.0, ORC_BITS) - 1.0;
    for (int64_t i = 0; i < n; i++)
        for (int d = 0; d < 3; d++) {
            double u = floor((x[3 * i + d] - lo[d]) * scale);
            if (u < 0.0) u = 0.0;
            if (u > qmax) u = qmax;
            q[3 * i + d] = (uint32_t)u;
        }
}

/* ------------------------------------------------------------------------- */
/* Octree over the key-sorted particles (Barnes & Hut 1986).  A cell is a    */
/* level and a 3*level-bit key prefix; its particles are a contiguous range.  */
/* A cell is split iff it holds more than n_leaf particles and is above the   */
/* deepest level.  Cells are stored in pre-order, children in key order.      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int level;
    int split;
    int64_t begin, end;
    int64_t first_child;   /* -1 if none */
    int64_t next_sibling;  /* -1 if last */
    int64_t node;          /* node number, -1 if fewer than two particles */
} orc_cell;

typedef struct {
    int64_t n;
    int n_leaf, n_crit;
    double theta;
    double lo[3], side;
    /* particles in new order */
    int64_t *perm;          /* perm[new] = old index */
    uint64_t *key;          /* sorted keys */
    double *x, *v, *a, *j, *m;  /* sorted copies (x at t_tree) */
    /* cells */
    orc_cell *cell;
    int64_t n_cell, cap_cell;
    /* nodes (cells with >= 2 particles), pre-order */
    int64_t n_node;
    int64_t *node_cell;
    double *nm, *nx, *nv, *na, *nj;
    /* groups */
    int64_t n_group;
    int64_t *group_cell;
    int64_t *group_first;   /* n_group + 1 */
    double *group_lo, *group_hi;
    /* lists */
    int64_t *list_off;      /* n_group + 1 */
    int32_t *entries;
    int64_t n_entries;
} orc_tree;

typedef struct { uint64_t key; int64_t idx; } orc_keyidx;

static int orc_cmp_keyidx(const void *pa, const void *pb)
{
    const orc_keyidx *a = (const orc_keyidx *)pa, *b = (const orc_keyidx *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

static int64_t orc_new_cell(orc_tree *t)
{
    if (t->n_cell == t->cap_cell) {
        t->cap_cell = t->cap_cell ? 2 * t->cap_cell : 1024;
        t->cell = (orc_cell *)realloc(t->cell, (size_t)t->cap_cell * sizeof(orc_cell));
    }
    return t->n_cell++;
}

static int64_t orc_build_cell(orc_tree *t, int level, int64_t b, int64_t e)
{
    int64_t id = orc_new_cell(t);
    orc_cell *c = &t->cell[id];
    c->level = level;
    c->begin = b;
    c->end = e;
    c->first_child = -1;
    c->next_sibling = -1;
    c->node = -1;
    c->split = (e - b > t->n_leaf) && (level < ORC_MAX_LEVEL);
    if (!c->split) return id;
    int shift = 3 * (ORC_MAX_LEVEL - level - 1);
    int64_t prev = -1;
    int64_t k = b;
    while (k < e) {
        uint64_t digit = (t->key[k] >> shift) & 7u;
        int64_t r = k + 1;
        while (r < e && ((t->key[r] >> shift) & 7u) == digit) r++;
        int64_t child = orc_build_cell(t, level + 1, k, r);
        if (prev < 0) t->cell[id].first_child = child;
        else t->cell[prev].next_sibling = child;
        prev = child;
        k = r;
    }
    return id;
}

/* Node moments (Section 2, step 1: tree nodes are pseudo-particles with       */
/* position, velocity, acceleration and its derivative).  READING: monopole  */
/* at the centre of mass, accumulated bottom-up as tree codes do.  A cell's  */
/* sums S = (sum m, sum m*x, sum m*v, sum m*a, sum m*jerk) start from zero;   */
/* a split cell adds its children's S in key order, an unsplit cell adds its */
/* particles' rounded products m_k*x_k in ascending order.  A node's mass is */
/* its sum of m, and X = (sum of m*x)/M, likewise for v, a and jerk, all at  */
/* the tree time.  One pass from the root visits every cell once.            */
static void orc_cell_sums(orc_tree *t, int64_t id, double s[13])
{
    const orc_cell *c = &t->cell[id];
    for (int q = 0; q < 13; q++) s[q] = 0.0;
    if (c->split) {
        for (int64_t ch = c->first_child; ch >= 0; ch = t->cell[ch].next_sibling) {
            double sc[13];
            orc_cell_sums(t, ch, sc);
            for (int q = 0; q < 13; q++) s[q] = s[q] + sc[q];
        }
    } else {
        for (int64_t k = c->begin; k < c->end; k++) {
            double mk = t->m[k];
            s[0] = s[0] + mk;
            for (int d = 0; d < 3; d++) {
                s[1 + d] = s[1 + d] + mk * t->x[3 * k + d];
                s[4 + d] = s[4 + d] + mk * t->v[3 * k + d];
                s[7 + d] = s[7 + d] + mk * t->a[3 * k + d];
                s[10 + d] = s[10 + d] + mk * t->j[3 * k + d];
            }
        }
    }
    if (c->node >= 0) {
        int64_t nd = c->node;
        t->nm[nd] = s[0];
        for (int d = 0; d < 3; d++) {
            t->nx[3 * nd + d] = s[1 + d] / s[0];
            t->nv[3 * nd + d] = s[4 + d] / s[0];
            t->na[3 * nd + d] = s[7 + d] / s[0];
            t->nj[3 * nd + d] = s[10 + d] / s[0];
        }
    }
}

/* Groups (modified tree algorithm of Barnes 1990, Section 2): walking the    */
/* tree in pre-order, the first cell with at most n_crit particles (or that   */
/* cannot be split) becomes a group; its particles share one list.            */
static void orc_find_groups(orc_tree *t, int64_t id, int64_t *count_only)
{
    const orc_cell *c = &t->cell[id];
    if (c->end - c->begin <= t->n_crit || !c->split) {
        if (count_only) { (*count_only)++; return; }
        int64_t g = t->n_group++;
        t->group_cell[g] = id;
        t->group_first[g] = c->begin;
        return;
    }
    for (int64_t ch = c->first_child; ch >= 0; ch = t->cell[ch].next_sibling)
        orc_find_groups(t, ch, count_only);
}

typedef struct { int32_t *e; int64_t n, cap; } orc_vec;

static void orc_push(orc_vec *v, int32_t x)
{
    if (v->n == v->cap) {
        v->cap = v->cap ? 2 * v->cap : 256;
        v->e = (int32_t *)realloc(v->e, (size_t)v->cap * sizeof(int32_t));
    }
    v->e[v->n++] = x;
}

/* Traversal for one group (Section 2, step 1: interaction list = the         */
/* group's own and nearby particles plus the accepted nodes).  READING of the */
/* opening test (Barnes-Hut with the group's bounding box): a cell whose     */
/* particle range overlaps the group is never accepted; otherwise a node is  */
/* accepted iff side_l^2 < theta^2 * d^2, d = distance from its centre of     */
/* mass to the group box; cells that are not accepted are opened, and         */
/* unsplit cells contribute their particles.                                  */
static void orc_walk(const orc_tree *t, int64_t id, int64_t gb, int64_t ge, const double blo[3],
                     const double bhi[3], double theta2, orc_vec *out)
{
    const orc_cell *c = &t->cell[id];
    int64_t cnt = c->end - c->begin;
    if (c->begin < ge && gb < c->end) {
        if (c->split) {
            for (int64_t ch = c->first_child; ch >= 0; ch = t->cell[ch].next_sibling)
                orc_walk(t, ch, gb, ge, blo, bhi, theta2, out);
        } else {
            for (int64_t k = c->begin; k < c->end; k++) orc_push(out, (int32_t)k);
        }
        return;
    }
    if (cnt == 1) {
        orc_push(out, (int32_t)c->begin);
        return;
    }
    const double *X = &t->nx[3 * c->node];
    double gap[3];
    for (int d = 0; d < 3; d++) {
        double g1 = blo[d] - X[d];
        double g2 = X[d] - bhi[d];
        double g = g1 > g2 ? g1 : g2;
        gap[d] = g > 0.0 ? g : 0.0;
    }
    double d2 = (gap[0] * gap[0] + gap[1] * gap[1]) + gap[2] * gap[2];
    double s = ldexp(t->side, -c->level);
    if (s * s < theta2 * d2) {
        orc_push(out, (int32_t)(t->n + c->node));
        return;
    }
    if (c->split) {
        for (int64_t ch = c->first_child; ch >= 0; ch = t->cell[ch].next_sibling)
            orc_walk(t, ch, gb, ge, blo, bhi, theta2, out);
    } else {
        for (int64_t k = c->begin; k < c->end; k++) orc_push(out, (int32_t)k);
    }
}

/* Build everything done at a tree time (Section 2, step 1).  Inputs are the  */
/* particles in their current order (x, v, a, jerk at the tree time); the     */
/* new order is the stable sort by (key, current index).                      */
orc_tree *orc_tree_build(int64_t n, const double *x, const double *v, const double *a,
                         const double *jerk, const double *m, int n_leaf, int n_crit, double theta)
{
    if (n < 1 || n_leaf < 1 || n_crit < 1) return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->n = n;
    t->n_leaf = n_leaf;
    t->n_crit = n_crit;
    t->theta = theta;
    orc_root_box(n, x, t->lo, &t->side);
    uint32_t *q = (uint32_t *)malloc((size_t)n * 3 * sizeof(uint32_t));
    orc_quantize(n, x, t->lo, t->side, q);
    orc_keyidx *ki = (orc_keyidx *)malloc((size_t)n * sizeof(orc_keyidx));
    for (int64_t i = 0; i < n; i++) {
        ki[i].key = orc_hilbert_key(q[3 * i], q[3 * i + 1], q[3 * i + 2]);
        ki[i].idx = i;
    }
    free(q);
    qsort(ki, (size_t)n, sizeof(orc_keyidx), orc_cmp_keyidx);
    t->perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    t->key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    t->x = (double *)malloc((size_t)n * 3 * sizeof(double));
    t->v = (double *)malloc((size_t)n * 3 * sizeof(double));
    t->a = (double *)malloc((size_t)n * 3 * sizeof(double));
    t->j = (double *)malloc((size_t)n * 3 * sizeof(double));
    t->m = (double *)malloc((size_t)n * sizeof(double));
    for (int64_t k = 0; k < n; k++) {
        int64_t o = ki[k].idx;
        t->perm[k] = o;
        t->key[k] = ki[k].key;
        t->m[k] = m[o];
        for (int d = 0; d < 3; d++) {
            t->x[3 * k + d] = x[3 * o + d];
            t->v[3 * k + d] = v[3 * o + d];
            t->a[3 * k + d] = a[3 * o + d];
            t->j[3 * k + d] = jerk[3 * o + d];
        }
    }
    free(ki);
    orc_build_cell(t, 0, 0, n);
    /* nodes: cells with at least two particles, pre-order */
    t->n_node = 0;
    for (int64_t c = 0; c < t->n_cell; c++)
        if (t->cell[c].end - t->cell[c].begin >= 2) t->cell[c].node = t->n_node++;
    t->node_cell = (int64_t *)malloc((size_t)(t->n_node + 1) * sizeof(int64_t));
    for (int64_t c = 0; c < t->n_cell; c++)
        if (t->cell[c].node >= 0) t->node_cell[t->cell[c].node] = c;
    size_t nn = (size_t)(t->n_node + 1);
    t->nm = (double *)malloc(nn * sizeof(double));
    t->nx = (double *)malloc(nn * 3 * sizeof(double));
    t->nv = (double *)malloc(nn * 3 * sizeof(double));
    t->na = (double *)malloc(nn * 3 * sizeof(double));
    t->nj = (double *)malloc(nn * 3 * sizeof(double));
    {
        double s_root[13];
        orc_cell_sums(t, 0, s_root);
    }
    /* groups */
    int64_t ng = 0;
    orc_find_groups(t, 0, &ng);
    t->group_cell = (int64_t *)malloc((size_t)ng * sizeof(int64_t));
    t->group_first = (int64_t *)malloc((size_t)(ng + 1) * sizeof(int64_t));
    t->n_group = 0;
    orc_find_groups(t, 0, NULL);
    t->group_first[ng] = n;
    t->group_lo = (double *)malloc((size_t)ng * 3 * sizeof(double));
    t->group_hi = (double *)malloc((size_t)ng * 3 * sizeof(double));
    for (int64_t g = 0; g < ng; g++) {
        int64_t b = t->group_first[g], e = t->group_first[g + 1];
        for (int d = 0; d < 3; d++) {
            double lo = t->x[3 * b + d], hi = lo;
            for (int64_t k = b + 1; k < e; k++) {
                double c = t->x[3 * k + d];
                if (c < lo) lo = c;
                if (c > hi) hi = c;
            }
            t->group_lo[3 * g + d] = lo;
            t->group_hi[3 * g + d] = hi;
        }
    }
    /* lists */
    orc_vec *lists = (orc_vec *)calloc((size_t)ng, sizeof(orc_vec));
    const double theta2 = theta * theta;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t g = 0; g < ng; g++)
        orc_walk(t, 0, t->group_first[g], t->group_first[g + 1], &t->group_lo[3 * g],
                 &t->group_hi[3 * g], theta2, &lists[g]);
    t->list_off = (int64_t *)malloc((size_t)(ng + 1) * sizeof(int64_t));
    t->list_off[0] = 0;
    for (int64_t g = 0; g < ng; g++) t->list_off[g + 1] = t->list_off[g] + lists[g].n;
    t->n_entries = t->list_off[ng];
    t->entries = (int32_t *)malloc((size_t)(t->n_entries + 1) * sizeof(int32_t));
    for (int64_t g = 0; g < ng; g++) {
        if (lists[g].n) memcpy(t->entries + t->list_off[g], lists[g].e, (size_t)lists[g].n * sizeof(int32_t));
        free(lists[g].e);
    }
    free(lists);
    return t;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    free(t->perm); free(t->key); free(t->x); free(t->v); free(t->a); free(t->j); free(t->m);
    free(t->cell); free(t->node_cell);
    free(t->nm); free(t->nx); free(t->nv); free(t->na); free(t->nj);
    free(t->group_cell); free(t->group_first); free(t->group_lo); free(t->group_hi);
    free(t->list_off); free(t->entries);
    free(t);
}

void orc_tree_sizes(const orc_tree *t, int64_t *n_node, int64_t *n_group, int64_t *n_entries,
                    int64_t *n_cell)
{
    *n_node = t->n_node;
    *n_group = t->n_group;
    *n_entries = t->n_entries;
    *n_cell = t->n_cell;
}

void orc_tree_root(const orc_tree *t, double lo[3], double *side)
{
    for (int d = 0; d < 3; d++) lo[d] = t->lo[d];
    *side = t->side;
}

/* Copy out.  Any pointer may be NULL to skip that array. */
void orc_tree_get(const orc_tree *t, int64_t *perm, uint64_t *keys, double *node_m, double *node_x,
                  double *node_v, double *node_a, double *node_j, int32_t *node_level,
                  int64_t *node_begin, int64_t *node_end, int64_t *group_first,
                  int64_t *list_off, int32_t *entries)
{
    int64_t M = t->n_node, G = t->n_group;
    if (perm) memcpy(perm, t->perm, (size_t)t->n * sizeof(int64_t));
    if (keys) memcpy(keys, t->key, (size_t)t->n * sizeof(uint64_t));
    if (node_m) memcpy(node_m, t->nm, (size_t)M * sizeof(double));
    if (node_x) memcpy(node_x, t->nx, (size_t)M * 3 * sizeof(double));
    if (node_v) memcpy(node_v, t->nv, (size_t)M * 3 * sizeof(double));
    if (node_a) memcpy(node_a, t->na, (size_t)M * 3 * sizeof(double));
    if (node_j) memcpy(node_j, t->nj, (size_t)M * 3 * sizeof(double));
    for (int64_t nd = 0; nd < M; nd++) {
        const orc_cell *c = &t->cell[t->node_cell[nd]];
        if (node_level) node_level[nd] = c->level;
        if (node_begin) node_begin[nd] = c->begin;
        if (node_end) node_end[nd] = c->end;
    }
    if (group_first) memcpy(group_first, t->group_first, (size_t)(G + 1) * sizeof(int64_t));
    if (list_off) memcpy(list_off, t->list_off, (size_t)(G + 1) * sizeof(int64_t));
    if (entries) memcpy(entries, t->entries, (size_t)t->n_entries * sizeof(int32_t));
}

/* ------------------------------------------------------------------------- */
/* Predictor (Section 2, steps 4 and 5: GRAPE predicts j-particles and nodes, */
/* the host predicts i-particles; 4th-order Hermite scheme of Makino &        */
/* Aarseth 1992): Taylor series to the jerk, dt = t - t0.                     */
/*   x_p = x + dt (v + dt/2 (a + dt/3 jerk)),  v_p = v + dt (a + dt/2 jerk)   */
/* ------------------------------------------------------------------------- */
void orc_predict(int64_t n, double t, const double *t0, const double *x, const double *v,
                 const double *a, const double *jerk, double *xp, double *vp)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        double dt = t - t0[i];
        double h2 = dt * 0.5, h3 = dt / 3.0;
        for (int d = 0; d < 3; d++) {
            int64_t k = 3 * i + d;
            xp[k] = x[k] + dt * (v[k] + h2 * (a[k] + h3 * jerk[k]));
            vp[k] = v[k] + dt * (a[k] + h2 * jerk[k]);
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Pairwise acceleration, jerk and potential with Plummer softening (the      */
/* force GRAPE computes, Section 2 step 5; 4th-order Hermite quantities):     */
/*   r = x_j - x_i, w = v_j - v_i, s = r.r + eps^2                            */
/*   a    += m r s^-3/2                                                       */
/*   jerk += m (w s^-3/2 - 3 (r.w) r s^-5/2)                                  */
/*   pot  -= m s^-1/2                                                         */
/* ------------------------------------------------------------------------- */
static void orc_pair(const double *xi, const double *vi, const double *xj, const double *vj,
                     double mj, double eps2, double acc[3], double jrk[3], double *pot)
{
    double r[3], w[3];
    for (int d = 0; d < 3; d++) { r[d] = xj[d] - xi[d]; w[d] = vj[d] - vi[d]; }
    double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
    double rinv = 1.0 / sqrt(s);
    double rinv2 = rinv * rinv;
    double mr3 = mj * rinv * rinv2;
    double rw = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
    double alpha = 3.0 * rw * rinv2;
    for (int d = 0; d < 3; d++) {
        acc[d] += mr3 * r[d];
        jrk[d] += mr3 * (w[d] - alpha * r[d]);
    }
    *pot -= mj * rinv;
}

static int64_t orc_group_of(int64_t i, int64_t n_group, const int64_t *group_first)
{
    int64_t lo = 0, hi = n_group;   /* group_first[lo] <= i < group_first[hi] */
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) / 2;
        if (group_first[mid] <= i) lo = mid; else hi = mid;
    }
    return lo;
}

/* Force over the interaction list of each active particle's group (Section  */
/* 2, steps 4a and 5).  xp, vp, m cover the combined memory (particles then   */
/* nodes); the i-particle is the predicted particle of the same index and is  */
/* skipped when it meets itself in the list (READING: self excluded).         */
/* Entries are summed in list order.                                          */
void orc_force_list(int64_t n_active, const int32_t *active, const double *xp, const double *vp,
                    const double *m, double eps2, int64_t n_group, const int64_t *group_first,
                    const int64_t *list_off, const int32_t *entries, double *acc, double *jerk,
                    double *pot)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_active; k++) {
        int64_t i = active[k];
        int64_t g = orc_group_of(i, n_group, group_first);
        double a3[3] = {0, 0, 0}, j3[3] = {0, 0, 0}, p = 0.0;
        for (int64_t e = list_off[g]; e < list_off[g + 1]; e++) {
            int64_t jj = entries[e];
            if (jj == i) continue;
            orc_pair(&xp[3 * i], &vp[3 * i], &xp[3 * jj], &vp[3 * jj], m[jj], eps2, a3, j3, &p);
        }
        for (int d = 0; d < 3; d++) { acc[3 * k + d] = a3[d]; jerk[3 * k + d] = j3[d]; }
        pot[k] = p;
    }
}

/* Direct summation over all particles 0..n-1 (the original Hermite scheme on */
/* GRAPE, Section 2 steps 1-7), same pair formula and ascending order.        */
void orc_force_direct(int64_t n_active, const int32_t *active, int64_t n, const double *xp,
                      const double *vp, const double *m, double eps2, double *acc, double *jerk,
                      double *pot)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < n_active; k++) {
        int64_t i = active[k];
        double a3[3] = {0, 0, 0}, j3[3] = {0, 0, 0}, p = 0.0;
        for (int64_t jj = 0; jj < n; jj++) {
            if (jj == i) continue;
            orc_pair(&xp[3 * i], &vp[3 * i], &xp[3 * jj], &vp[3 * jj], m[jj], eps2, a3, j3, &p);
        }
        for (int d = 0; d < 3; d++) { acc[3 * k + d] = a3[d]; jerk[3 * k + d] = j3[d]; }
        pot[k] = p;
    }
}

/* ------------------------------------------------------------------------- */
/* Hermite corrector (Makino & Aarseth 1992, cited in Section 1; step 6).    */
/* With D = t1 - t0 and (a0, j0) at t0, (a1, j1) at t1:                       */
/*   a2 = (-6 (a0 - a1) - D (4 j0 + 2 j1)) / D^2      (second derivative, t0) */
/*   a3 = (12 (a0 - a1) + 6 D (j0 + j1)) / D^3        (third derivative)      */
/*   x1 = x_p + a2 D^4/24 + a3 D^5/120,  v1 = v_p + a2 D^3/6 + a3 D^4/24      */
/* The new step follows Aarseth's criterion with eta (Section 3):            */
/*   dt = sqrt(eta (|a1||a2'| + |j1|^2) / (|j1||a3| + |a2'|^2)),  a2' = a2+D a3 */
/* ------------------------------------------------------------------------- */
static double orc_norm3(const double *u) { return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

void orc_correct(int64_t n_active, double t1, const double *t0, const double *xp, const double *vp,
                 const double *a0, const double *j0, const double *a1, const double *j1, double eta,
                 double *x_out, double *v_out, double *dt_aarseth)
{
    for (int64_t k = 0; k < n_active; k++) {
        double D = t1 - t0[k];
        double D2 = D * D, D3 = D2 * D;
        double a2[3], a3[3], a2n[3];
        for (int d = 0; d < 3; d++) {
            int64_t q = 3 * k + d;
            double da = a0[q] - a1[q];
            a2[d] = (-6.0 * da - D * (4.0 * j0[q] + 2.0 * j1[q])) / D2;
            a3[d] = (12.0 * da + 6.0 * D * (j0[q] + j1[q])) / D3;
            x_out[q] = xp[q] + a2[d] * (D2 * D2 / 24.0) + a3[d] * (D2 * D3 / 120.0);
            v_out[q] = vp[q] + a2[d] * (D3 / 6.0) + a3[d] * (D2 * D2 / 24.0);
            a2n[d] = a2[d] + D * a3[d];
        }
        double na = orc_norm3(&a1[3 * k]), nj = orc_norm3(&j1[3 * k]);
        double n2 = orc_norm3(a2n), n3 = orc_norm3(a3);
        double num = na * n2 + nj * nj;
        double den = nj * n3 + n2 * n2;
        dt_aarseth[k] = den > 0.0 ? sqrt(eta * num / den) : INFINITY;
    }
}

/* Block timestep (McMillan 1986, Section 1).  READING: the largest power of  */
/* two h <= min(dt, dt_tree, 2 dt_old) such that t1 is a multiple of h; the   */
/* tree interval caps every step (Section 2).  dt_old <= 0 means no previous  */
/* step.  Returns 0 if h would fall below 2^-40.                              */
double orc_block_step(double dt, double t1, double dt_tree, double dt_old)
{
    double cap = dt < dt_tree ? dt : dt_tree;
    if (dt_old > 0.0 && 2.0 * dt_old < cap) cap = 2.0 * dt_old;
    if (!(cap > 0.0)) return 0.0;
    int e;
    frexp(cap, &e);
    double h = ldexp(1.0, e - 1);
    const double floor_h = ldexp(1.0, -40);
    while (h >= floor_h && fmod(t1, h) != 0.0) h *= 0.5;
    return h >= floor_h ? h : 0.0;
}

/* Total energy by direct summation (Section 3: the potential energy is       */
/* computed directly, not with the tree): K = sum m v^2 / 2,                 */
/* W = -sum_{i<j} m_i m_j / sqrt(r^2 + eps^2).                               */
void orc_energy(int64_t n, const double *x, const double *v, const double *m, double eps2,
                double *kin, double *pot)
{
    double *row = (double *)malloc((size_t)n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        double s = 0.0;
        for (int64_t j = i + 1; j < n; j++) {
            double dx = x[3 * j] - x[3 * i], dy = x[3 * j + 1] - x[3 * i + 1], dz = x[3 * j + 2] - x[3 * i + 2];
            s += m[j] / sqrt(dx * dx + dy * dy + dz * dz + eps2);
        }
        row[i] = m[i] * s;
    }
    double W = 0.0, K = 0.0;
    for (int64_t i = 0; i < n; i++) {
        W -= row[i];
        K += 0.5 * m[i] * (v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2]);
    }
    free(row);
    *kin = K;
    *pot = W;
}

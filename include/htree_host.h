/*
 * htree_host — host side of the tree/Hermite scheme: the tree, groups and
 * interaction lists built at every multiple of the tree interval (Fukushige &
 * Kawai, Section 2, step 1), and the host's Hermite corrector and block
 * timestep selection (steps 2, 6 and 7).  Multithreaded with OpenMP; results
 * do not depend on the thread count.
 *
 * Tree: particles are sorted by their 63-bit Peano-Hilbert key (21 bits per
 * axis, root cube of power-of-two side at the componentwise minimum), ties
 * by current index.  Cells split while they hold more than n_leaf particles
 * (down to level 21).  Nodes are the cells with at least two particles, in
 * pre-order; node k is combined index N + k and carries total mass and the
 * mass-weighted mean of position, velocity, acceleration and jerk, summed
 * bottom-up: a cell's sums (m, m x, m v, m a, m jerk) start from zero and
 * add, for a split cell, its children's sums in key order, otherwise its
 * particles' rounded products in ascending order (no fused multiply-add);
 * the means are these sums divided by the mass sum.  Groups
 * are the first cells on every root-to-leaf path with at most n_crit
 * particles (or that cannot split).  A group's list holds, in pre-order, the
 * nodes that pass the opening test  side^2 < theta^2 d^2  (d = distance from
 * the node's centre of mass to the group's bounding box; nodes overlapping
 * the group never pass) and the particles of every leaf reached otherwise.
 *
 * Conventions: return 0 on success, negative on bad arguments (-1) or
 * allocation failure (-3); vectors are row-major [n][3] doubles; the caller
 * owns every array passed in; htb_* objects are freed with htb_free.
 */
#ifndef HTREE_HOST_H
#define HTREE_HOST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct htb_tree htb_tree;

/* Build keys, tree, node moments, groups and lists for particles in their
 * current order (x, v, a, jerk valid at the tree time). */
int htb_build(htb_tree **out, int64_t n, const double *x, const double *v, const double *a,
              const double *jerk, const double *m, int32_t n_leaf, int32_t n_crit, double theta);

int htb_sizes(const htb_tree *t, int64_t *n_node, int64_t *n_group, int64_t *n_entries);

/* Copy results out; any pointer may be NULL.  perm[new] = old index;
 * node arrays have n_node rows; group_first and list_off have n_group+1. */
int htb_get(const htb_tree *t, int64_t *perm, uint64_t *keys, double *node_m, double *node_x,
            double *node_v, double *node_a, double *node_j, int32_t *node_level, int64_t *node_begin,
            int64_t *node_end, int64_t *group_first, int64_t *list_off, int32_t *entries);

void htb_free(htb_tree *t);

/* Peano-Hilbert keys of integer coordinates q[n][3] (each < 2^21). */
int htb_hilbert_keys(int64_t n, const uint32_t *q, uint64_t *keys);

/* Step 2: the next block time min(t0 + dt) and the particles due then, in
 * ascending order.  active must hold n entries; *n_active receives the count. */
int htb_next_block(int64_t n, const double *t0, const double *dt, double *t_next, int32_t *active,
                   int64_t *n_active);

/* Step 6 for the active particles: Hermite corrector from (a0, jerk0) at t0
 * to (acc1, jerk1) at t1, then Aarseth's step with eta, quantised to the
 * largest power of two <= min(step, dt_tree, 2 dt_old) of which t1 is a
 * multiple.  Updates x, v, a, jerk, t0, dt of particles ids[] in place.
 * Returns -2 if a step would fall below 2^-40. */
int htb_correct(int64_t n_active, const int32_t *ids, double t1, double eta, double dt_tree, double *t0,
                double *dt, double *x, double *v, double *a, double *jerk, const double *acc1,
                const double *jerk1);

/* Initial block steps from eta |a| / |jerk| (capped by dt_tree) at t = 0. */
int htb_initial_steps(int64_t n, double eta, double dt_tree, const double *a, const double *jerk, double *dt);

/* ---------------------------------------------------------------------------
 * The same host steps for many clusters at once (batched engine): one call,
 * OpenMP across clusters.  Each cluster is described by the caller's arrays
 * (particles in tree order); the library only reads and writes through them.
 */
typedef struct {
    int64_t n;          /* particles */
    double eta;         /* Aarseth accuracy parameter */
    double dt_tree;     /* tree interval (largest block step) */
    double *t0, *dt;    /* [n] time of data, block step */
    double *x, *v, *a, *jerk;   /* [n][3] */
    const double *m;    /* [n] */
    double *pot;        /* [n] last potential */
    int32_t *active;    /* [n] scratch: active ids of the current step */
    int64_t n_active;   /* out of htb_next_block_many */
    double t_next;      /* out of htb_next_block_many */
} htb_cluster;

/* Step 2 for every cluster: t_next, n_active and active[] of each. */
int htb_next_block_many(int32_t n_clusters, htb_cluster *cl);

/* Step 6 for every cluster's current active set (from htb_next_block_many):
 * forces of cluster k are rows off[k] .. off[k] + n_active - 1 of acc [*][3],
 * jerk [*][3] and pot [*].  Then, unless the cluster has reached a tree time
 * (t_next a multiple of dt_tree, where it must rebuild), its corrected
 * particles are written as 120-byte update rows (layout of ht_row in htree.h:
 * int32 idx, int32 pad, double t0, m, x[3], v[3], a[3], jerk[3]) at
 * rows + row_off[k].  rebuild[k] is set to 1 for clusters at a tree time.
 * Returns -2 if a step would fall below 2^-40. */
int htb_correct_many(int32_t n_clusters, htb_cluster *cl, const int64_t *off, const double *acc,
                     const double *jerk, const double *pot, const int64_t *row_off, void *rows,
                     int32_t *rebuild);

#ifdef __cplusplus
}
#endif
#endif /* HTREE_HOST_H */

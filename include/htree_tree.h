/*
 * htree_tree — step 1 of the tree/Hermite scheme on the device (Fukushige &
 * Kawai, Section 2, step 1: the tree, the node data and the interaction
 * lists, rebuilt at every multiple of the tree interval; the paper builds them
 * on the host, and its Section 3 notes that the tree time per particle step
 * grows as the tree interval shrinks).
 *
 * The definitions are those of the host builder (include/htree_host.h) and
 * the results are bit-identical to its results: keys, particle order, node
 * moments, node levels and ranges, groups, list offsets and list entries.
 *
 *   - particles: 63-bit Peano-Hilbert keys (21 bits per axis, root cube of
 *     power-of-two side at the componentwise minimum), stable sort by
 *     (key, current index);
 *   - cells split while they hold more than n_leaf particles (down to level
 *     21); nodes are the cells with at least two particles, in pre-order, and
 *     carry total mass and mass-weighted means of x, v, a, jerk, summed
 *     bottom-up (a split cell adds its children's sums in key order, a leaf
 *     its particles' rounded products in ascending order);
 *   - groups are the first cells on each root-to-leaf path with at most
 *     n_crit particles (or that cannot split);
 *   - a group's list holds, in pre-order, the nodes with side^2 < theta^2 d^2
 *     (d from the node's centre of mass to the group's bounding box; nodes
 *     that overlap the group never pass) and the particles of every leaf
 *     reached otherwise.  Entries are combined indices: particle k (key
 *     order) is k, node q is n + q.
 *
 * Conventions: return 0 on success or a negative status (values as
 * ht_status in htree.h); htd_last_error() then holds a message for this
 * thread.  Device arrays are row-major [n][3] doubles for vectors.  The
 * library owns every array of the tree object; the caller owns the input
 * arrays and every host array passed in.  Calls on one object are not
 * thread-safe.  htd_build is synchronous with the object's stream.
 */
#ifndef HTREE_TREE_H
#define HTREE_TREE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HTD_OK = 0, HTD_EINVAL = -1, HTD_ERANGE = -2, HTD_ENOMEM = -3, HTD_ESTATE = -4, HTD_EHIP = -5 };

typedef struct htd_tree htd_tree;

/* Device pointers to the last build's results (owned by the tree object,
 * valid until the next build or htd_destroy).  x .. m are the particles in
 * key order; node vectors have n_node rows; group_first and list_off have
 * n_group + 1 entries. */
typedef struct {
    const int64_t *perm;        /* perm[new] = old index */
    const uint64_t *keys;       /* sorted keys */
    const double *x, *v, *a, *jerk, *m;
    const double *node_m, *node_x, *node_v, *node_a, *node_j;
    const int64_t *group_first, *list_off;
    const int32_t *entries;
} htd_view;

/* A builder for up to n_max particles (1 <= n_max <= 2^26) on `device`,
 * working on `stream` (a hipStream_t; NULL = the default stream).  Device
 * memory for the particle-sized arrays is allocated here; arrays whose size
 * depends on the tree grow on demand inside htd_build. */
int htd_create(htd_tree **out, int32_t device, void *stream, int64_t n_max);
int htd_destroy(htd_tree *t);

/* Build from n particles in device memory (x, v, a, jerk [n][3], m [n], valid
 * at the tree time).  HTD_EINVAL for n outside [1, n_max], NULL arrays,
 * n_leaf or n_crit < 1, or theta negative or not finite; HTD_ENOMEM if a
 * growing array cannot be allocated. */
int htd_build(htd_tree *t, int64_t n, const double *d_x, const double *d_v, const double *d_a,
              const double *d_jerk, const double *d_m, int32_t n_leaf, int32_t n_crit, double theta);

/* Sizes of the last build (HTD_ESTATE before a successful build). */
int htd_sizes(const htd_tree *t, int64_t *n_node, int64_t *n_group, int64_t *n_entries, int64_t *n_cell);

/* Root cube of the last build: lower corner lo[3] and side. */
int htd_root(const htd_tree *t, double *lo, double *side);

/* Copy the last build's results into host arrays, as htb_get does; any
 * pointer may be NULL.  Synchronous. */
int htd_get(const htd_tree *t, int64_t *perm, uint64_t *keys, double *node_m, double *node_x, double *node_v,
            double *node_a, double *node_j, int32_t *node_level, int64_t *node_begin, int64_t *node_end,
            int64_t *group_first, int64_t *list_off, int32_t *entries);

/* Device pointers to the last build's results. */
int htd_device_view(const htd_tree *t, htd_view *out);

/* Device time of the last build's phases in ms: keys, sort, cells (with the
 * size read-back), moments, lists, CSR assembly, and the total. ms[7]. */
int htd_phase_ms(const htd_tree *t, double *ms);

/* Device bytes the builder holds now (its arrays grow with the largest tree
 * built so far), for admission by device footprint. */
int htd_device_bytes(const htd_tree *t, size_t *bytes);

const char *htd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HTREE_TREE_H */

/*
 * htree — block-step force evaluation of the tree/Hermite scheme on gfx950.
 *
 * Operation (Fukushige & Kawai, Section 2, tree-Hermite steps 1, 4a and 5):
 * the host builds, at every multiple of the tree interval, a tree whose nodes
 * are pseudo-particles (mass, centre-of-mass position, velocity, acceleration
 * and jerk), groups of neighbouring particles, and one interaction list per
 * group.  Particles and nodes live in one combined memory: indices [0, N) are
 * particles, [N, N+M) are nodes.  At every block step the caller updates the
 * corrected particles (step 6), predicts the whole memory to the block time
 * (step 5, predictor of the 4th-order Hermite scheme), and asks for the
 * acceleration, jerk and potential of the active particles, each summed over
 * the list of its group (steps 4a and 5).  ht_force_direct sums over all
 * particles instead (the original Hermite scheme, same section).
 *
 * Pair interaction with Plummer softening (r = x_j - x_i, w = v_j - v_i,
 * s = r.r + eps^2):  a += m r s^-3/2;  jerk += m (w s^-3/2 - 3 (r.w) r s^-5/2);
 * pot -= m s^-1/2.  A particle never interacts with itself.
 *
 * Precision forms:
 *   HT_PREC_FP64  — everything in FP64.
 *   HT_PREC_MIXED — the j-memory stores m, a and jerk in FP32 (times,
 *                   positions and velocities in FP64); s^-1/2 starts from
 *                   the FP32 reciprocal square root, refined by one Newton
 *                   step in FP64 (relative error about 1e-13); prediction,
 *                   x_j - x_i, the pair terms and every sum are FP64.  (With
 *                   s^-3/2 and the jerk terms in FP32, particles whose jerk
 *                   terms cancel to a few hundredths of their size missed
 *                   the 1e-5 jerk tolerance.)
 *
 * Conventions for every entry point:
 *   - Return HT_OK (0) or a negative ht_status; ht_last_error() then holds a
 *     message for the calling thread.  Arguments are validated before any
 *     device work is queued; on error nothing is modified.
 *   - Update rows whose particle indices sit in device memory (the *_async
 *     updates, ht_step_async, ht_step_graph) cannot be checked before the
 *     launch: the kernel drops every row whose index is outside [0, N),
 *     writes the other rows, and the next call that synchronises the
 *     context's stream (ht_sync, ht_force, ht_state_get, ht_dev_next_block,
 *     ...) returns HT_ERANGE once for them.  Batched row updates are checked
 *     the same way and reported by ht_batch_sync or ht_batch_dev_next_block.
 *   - Host arrays belong to the caller and are never retained after return.
 *     Vectors are row-major [n][3] doubles.
 *   - Device memory for the context is one workspace, either supplied by the
 *     caller (any device allocation of at least ht_workspace_bytes() bytes,
 *     256-byte aligned) or allocated by the library when NULL is passed.
 *   - Work is queued on the context's stream.  Calls that return results to
 *     host arrays synchronise that stream; *_async calls do not.
 *   - A context is not thread-safe; distinct contexts may be used from
 *     distinct threads.
 */
#ifndef HTREE_H
#define HTREE_H

#include <stddef.h>
#include <stdint.h>

#include "htree_tree.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ht_ctx ht_ctx;

typedef enum {
    HT_OK = 0,
    HT_EINVAL = -1,  /* malformed argument (sizes, order, NULL, duplicates) */
    HT_ERANGE = -2,  /* index outside the valid range or over a capacity   */
    HT_ENOMEM = -3,  /* allocation failed                                   */
    HT_ESTATE = -4,  /* call out of order (e.g. force before lists/predict) */
    HT_EHIP = -5     /* HIP runtime error; message names it                 */
} ht_status;

typedef enum { HT_PREC_FP64 = 0, HT_PREC_MIXED = 1 } ht_precision;

/* How ht_predict is carried out.  FUSED: ht_predict only records t and each
 * force kernel predicts every j-particle and node it gathers, in registers.
 * EAGER: ht_predict runs a kernel that predicts the whole combined memory
 * into separate arrays that force kernels then read. */
typedef enum { HT_PREDICT_FUSED = 0, HT_PREDICT_EAGER = 1 } ht_predict_mode;

typedef struct {
    int32_t device;        /* HIP device ordinal                                 */
    int32_t precision;     /* ht_precision                                       */
    int32_t predict_mode;  /* ht_predict_mode                                    */
    int32_t n_max;         /* capacity: particles                                */
    int32_t node_max;      /* capacity: tree nodes                               */
    int32_t group_max;     /* capacity: groups (= interaction lists)             */
    int64_t list_max;      /* capacity: total list entries over all groups      */
    int32_t active_max;    /* capacity: active particles per force call         */
    double eps2;           /* softening length squared (>= 0)                    */
    void *stream;          /* hipStream_t to queue on; NULL = library's own      */
} ht_config;

/* Bytes of device workspace a context with this configuration needs. */
int ht_workspace_bytes(const ht_config *cfg, size_t *bytes);

/* Create a context.  d_workspace may be NULL (library allocates) or a device
 * pointer of at least ht_workspace_bytes() bytes that outlives the context. */
int ht_create(ht_ctx **out, const ht_config *cfg, void *d_workspace, size_t workspace_bytes);
int ht_destroy(ht_ctx *ctx);

/* Step 1 / step 6: particles into j-memory.
 * idx == NULL: full upload of particles 0..n-1; sets N = n, and when N changes
 *              drops the nodes and lists (they must be set again).
 * idx != NULL: update particles idx[0..n-1] (each < N, no repeats).
 * t0[n]: time of each particle's data; m[n]; x, v, a, jerk: [n][3]. */
int ht_set_j_particles(ht_ctx *ctx, int32_t n, const int32_t *idx, const double *t0, const double *m,
                       const double *x, const double *v, const double *a, const double *jerk);

/* Same as ht_set_j_particles with idx != NULL, but every pointer is device
 * memory (same layouts) and the call is asynchronous on the stream. */
int ht_set_j_particles_async(ht_ctx *ctx, int32_t n, const int32_t *d_idx, const double *d_t0,
                             const double *d_m, const double *d_x, const double *d_v, const double *d_a,
                             const double *d_jerk);

/* Step 1: tree nodes as pseudo-particles at combined indices N..N+M-1, all
 * valid at t_tree.  m[M]; x, v, a, jerk: [M][3].  Invalidates the lists. */
int ht_set_nodes(ht_ctx *ctx, int32_t n_nodes, double t_tree, const double *m, const double *x,
                 const double *v, const double *a, const double *jerk);

/* Step 1: groups and their lists.  group_first[G+1] is a strictly increasing
 * cover of [0, N) (group g holds particles group_first[g]..group_first[g+1]-1);
 * list_off[G+1] is non-decreasing from 0; entries[list_off[G]] are combined
 * indices in [0, N+M).  Requires particles and nodes to be set. */
int ht_set_interaction_lists(ht_ctx *ctx, int32_t n_groups, const int64_t *group_first,
                             const int64_t *list_off, const int32_t *entries);

/* Form of the interaction lists in device memory.  CSR (the default): one
 * combined index per entry.  RUNS (Section 2's indirect addressing: a cell-
 * index memory of start and count pairs, each group's nodes copied
 * contiguously): at ht_set_interaction_lists every list's node entries are
 * replaced, in list order, by copies of their records at consecutive indices
 * from N + M on (library-owned device memory, 128 bytes per node entry), and
 * each list is stored as runs of consecutive indices; the force kernel
 * expands a round's runs in LDS.  The expanded lists are the CSR lists'
 * records in the same order, so every result is the CSR form's, bit for bit.
 * RUNS needs fused prediction and serves the single-context calls (ht_force,
 * ht_force_async, ht_step_async, ht_dev_step); batched calls, graph steps,
 * the device loops and device rebuilds take CSR only (HT_EINVAL).  Changing
 * the form drops the lists: set them again. */
typedef enum { HT_LISTS_CSR = 0, HT_LISTS_RUNS = 1, HT_LISTS_UNION = 2 } ht_list_form;
int ht_set_list_form(ht_ctx *ctx, int32_t form);

/* Union tiles (HT_LISTS_UNION).  Section 3, eq. (3): the force pipelines
 * lose efficiency when a group has few active particles; here a gathered
 * entry is shared among the active particles of several groups.  The lists
 * are kept as CSR;
 * at ht_set_interaction_lists the groups are also taken in runs of `width`
 * consecutive groups (consecutive in the space-filling order, so their lists
 * overlap), and each run gets the union of its members' lists (each entry
 * once, in order of first appearance over the members in group order) with
 * one bit per member whose own list holds the entry (library-owned device
 * memory, 5 bytes per union entry).  Per call the planner covers a run's
 * active particles either by the usual tiles of each group or by tiles over
 * the run's union list, whichever its cost model finds cheaper; in a union
 * tile a pair counts only where the entry's bit for the i-particle's group is
 * set, so every particle sums exactly its own list, in another order (results
 * agree with the CSR form to rounding, not bit for bit).  width: 2..8
 * (HT_EINVAL otherwise), default 4; changing it drops the lists.  Pairs
 * reported by ht_last_stats stay the list interactions.  Served calls as for
 * RUNS. */
int ht_set_union_width(ht_ctx *ctx, int32_t width);

/* Step 5 (predictor): predict particles and nodes to block time t. */
int ht_predict(ht_ctx *ctx, double t);

/* ht_predict(ctxs[k], t[k]) for k < n_ctx (arguments checked for all first). */
int ht_predict_many(int32_t n_ctx, ht_ctx *const *ctxs, const double *t);

/* Steps 4a and 5: acc, jerk ([n][3]) and pot ([n]) of the particles
 * active_ids[0..n-1] (strictly increasing, each < N), summed over their
 * groups' lists at the predicted time.  n_active == 0 is a no-op. */
int ht_force(ht_ctx *ctx, int32_t n_active, const int32_t *active_ids, double *acc, double *jerk,
             double *pot);

/* As ht_force with results written to device arrays, asynchronously.  The
 * work plan is packed into a pinned host slot (a ring of four, so the host can
 * run ahead of the device) that the device reads directly; a slot is reused
 * only after the launch that read it has completed. */
int ht_force_async(ht_ctx *ctx, int32_t n_active, const int32_t *active_ids, double *d_acc,
                   double *d_jerk, double *d_pot);

/* Direct summation over all N particles (nodes and lists unused). */
int ht_force_direct(ht_ctx *ctx, int32_t n_active, const int32_t *active_ids, double *acc, double *jerk,
                    double *pot);
int ht_force_direct_async(ht_ctx *ctx, int32_t n_active, const int32_t *active_ids, double *d_acc,
                          double *d_jerk, double *d_pot);

/* One block step in one call, asynchronously: the j-memory update of
 * ht_set_j_particles_async (n_upd rows, device arrays; n_upd = 0 skips it),
 * then ht_predict(t), then ht_force_async on active_ids (host array).  The
 * update and the delivery of the work plan share one launch. */
int ht_step_async(ht_ctx *ctx, int32_t n_upd, const int32_t *d_idx, const double *d_t0, const double *d_m,
                  const double *d_x, const double *d_v, const double *d_a, const double *d_jerk, double t,
                  int32_t n_active, const int32_t *active_ids, double *d_acc, double *d_jerk_out,
                  double *d_pot);

/* ht_step_async replayed through a HIP graph: the same arguments and the same
 * results, bit for bit.  The step's three launches (plan delivery with the
 * update, force, split reduction) are captured once per context into four
 * graphs (one per header slot, used in turn) whose kernels read the step's sizes from memory (a pinned header the
 * host rewrites before each replay, and the plan) and run on fixed grids, so
 * every replay is one hipGraphLaunch on the context's stream.  Needs
 * HT_PREDICT_FUSED; kernel timing (ht_set_timing) brackets the whole graph. */
int ht_step_graph(ht_ctx *ctx, int32_t n_upd, const int32_t *d_idx, const double *d_t0, const double *d_m,
                  const double *d_x, const double *d_v, const double *d_a, const double *d_jerk, double t,
                  int32_t n_active, const int32_t *active_ids, double *d_acc, double *d_jerk_out,
                  double *d_pot);

/* ---------------------------------------------------------------------------
 * Device-resident integration (steps 2 and 6 of Section 2 on the device; the
 * host keeps the tree, the lists and the work plan).
 *
 * ht_state_enable allocates the context's FP64 particle state on the device
 * (x, v, a, jerk [N][3], t0, dt, m, pot [N]).  ht_state_set uploads it from host
 * arrays (the layouts of ht_set_j_particles; pot may be NULL for zeros) and
 * rewrites the j-records; ht_state_get copies it back (any pointer may be NULL).
 *
 * ht_dev_next_block finds, on the device, the next block time t_next = min(t0 +
 * dt) and the particles due then (ascending), and returns them; *active points
 * into pinned memory owned by the context, valid until the next call.  It
 * synchronises with the stream, and fails with HT_ERANGE if the previous
 * step's corrector produced a block step below 2^-40.
 *
 * ht_dev_step then computes the force on that active set at t_next (as
 * ht_force_async), and on the device applies the Hermite corrector, Aarseth's
 * step with eta and the block quantisation (largest power of two <= min(step,
 * dt_tree, 2 dt_old) of which t_next is a multiple), writes the new state,
 * potential and j-records.  Asynchronous.  It gives the same bits as the host
 * corrector (htb_correct) given the same forces.  At a tree time the caller
 * either copies the state back, rebuilds on the host and uploads it again, or
 * calls ht_state_rebuild.
 *
 * ht_state_rebuild is step 1 on the device (Section 2, step 1) for a resident
 * state at a tree time t_tree (every particle synchronised there; the caller
 * guarantees it): the device tree builder t (include/htree_tree.h) builds
 * keys, order, tree, node moments, groups and lists from the resident x, v,
 * a, jerk, m; the state is reordered into the new key order (every t0 set to
 * t_tree), particle and node records are rewritten, and the new lists replace
 * the old ones.  perm (host, n entries, may be NULL) receives perm[new] = old.
 * The result is bit-identical to copying the state back, building with
 * htb_build and uploading it.  HT_ERANGE, with the context unchanged, if the
 * tree needs more nodes, groups or list entries than the context holds.
 * Synchronous. */
int ht_state_enable(ht_ctx *ctx);
/* Device bytes of the resident state of a context with this configuration,
 * and ht_state_enable on caller-owned device memory of at least that many
 * bytes (256-byte aligned, outliving the context), so that all of a
 * cluster's device memory can come from the caller's allocator.  Either form
 * also allocates 4 (n_max + 1) + 24 bytes of pinned host memory for the
 * scheduler's results. */
int ht_state_bytes(const ht_config *cfg, size_t *bytes);
int ht_state_enable_ws(ht_ctx *ctx, void *d_mem, size_t bytes);
int ht_state_set(ht_ctx *ctx, int32_t n, const double *t0, const double *dt, const double *m, const double *x,
                 const double *v, const double *a, const double *jerk, const double *pot);
int ht_state_get(ht_ctx *ctx, double *t0, double *dt, double *x, double *v, double *a, double *jerk, double *pot);
int ht_dev_next_block(ht_ctx *ctx, double *t_next, int64_t *n_active, const int32_t **active);
int ht_dev_step(ht_ctx *ctx, double eta, double dt_tree);
/* The same step for the direct Hermite scheme (Section 2's comparison): the
 * force on the active set over all N particles (as ht_force_direct_async);
 * needs no nodes or lists, and no rebuild at tree times. */
int ht_dev_step_direct(ht_ctx *ctx, double eta, double dt_tree);
/* Resident mode: up to max_steps block steps (Section 2, steps 2 and 4a-6)
 * queued back to back with no host round trip between them.  Each step runs
 * the scheduler, a device work planner that builds the host planner's work
 * items (so the forces, and the run, have the same bits as step-by-step
 * ht_dev_next_block + ht_dev_step), the force and reduce launches on fixed
 * grids, and the corrector.  The loop stops before the first block time after
 * t_stop, and after the step at t_stop (a tree time, where the caller
 * rebuilds).  Synchronises once, at the end; *steps, *t_last (block time of
 * the last step taken) and *particle_steps report what was done.  Needs fused
 * prediction and a whole-number gather cost (HT_EINVAL otherwise).
 * HT_ERANGE if a plan exceeded the context's capacity or a step fell below
 * 2^-40: the steps before it stand and the state is consistent. */
int ht_dev_run(ht_ctx *ctx, double eta, double dt_tree, double t_stop, int32_t max_steps, int32_t *steps,
               double *t_last, int64_t *particle_steps);
int ht_state_rebuild(ht_ctx *ctx, htd_tree *t, int32_t n_leaf, int32_t n_crit, double theta, double t_tree,
                     int64_t *perm);

/* Predicted position and velocity ([n][3]) of combined indices idx[0..n-1]
 * at the current block time, computed by the device predictor. */
int ht_get_predicted(ht_ctx *ctx, int32_t n, const int32_t *idx, double *xp, double *vp);

/* Force on the active particles of several contexts in one launch (the
 * batched block step).  All contexts must be on one device with one
 * precision, predicted, with lists set; results go to device arrays per
 * context.  Work is queued on ctxs[0]'s stream; each context's result is the
 * same as from its own ht_force_async call. */
int ht_force_batch_async(int32_t n_ctx, ht_ctx *const *ctxs, const int32_t *n_active,
                         const int32_t *const *active_ids, double *const *d_acc, double *const *d_jerk,
                         double *const *d_pot);

/* ---------------------------------------------------------------------------
 * Batched engine step (many clusters, one launch per phase).
 *
 * A batch owns device staging for the updates and work plans of all clusters
 * in one engine step.  Its contexts must share the batch's stream, device,
 * precision and predict mode; each keeps its own j-memory, lists and block
 * time (set by ht_predict on that context).  Work plans are made per context,
 * so every cluster gets bit-identical results alone and in any batch.
 * Capacities: max_clusters <= 1024 contexts per call; max_items work items and
 * max_active active particles summed over the contexts of one force call;
 * max_rows update rows summed over one update call.
 */
typedef struct ht_batch ht_batch;

/* One corrected particle for a j-memory update (step 6): row-major doubles. */
typedef struct {
    int32_t idx;     /* particle index in [0, N) of its context */
    int32_t pad;
    double t0;       /* time the data below refer to */
    double m;
    double x[3], v[3], a[3], jerk[3];
} ht_row;

int ht_batch_workspace_bytes(int32_t max_clusters, int64_t max_items, int64_t max_active, int64_t max_rows,
                             size_t *bytes);
/* stream must be the hipStream_t the contexts share; d_workspace as for ht_create. */
int ht_batch_create(ht_batch **out, int32_t device, void *stream, int32_t max_clusters, int64_t max_items,
                    int64_t max_active, int64_t max_rows, void *d_workspace, size_t workspace_bytes);
int ht_batch_destroy(ht_batch *b);

/* Step 6 for several contexts: rows[k][0..n_rows[k]-1] (host) go to ctxs[k]
 * (indices distinct within a context).  The rows are packed into pinned
 * staging and one kernel reads them from there and writes every context's
 * records (no separate copy); asynchronous; the contexts must be predicted
 * again afterwards. */
int ht_batch_update_async(ht_batch *b, int32_t n_ctx, ht_ctx *const *ctxs, const int32_t *n_rows,
                          const ht_row *const *rows);

/* As ht_batch_update_async, but the kernel reads the caller's rows in place:
 * each rows[k] must be pinned host memory (hipHostMalloc) and must stay
 * unchanged until the batch's stream has passed this call (for example until
 * the next ht_batch_sync).  Saves the copy into the batch's staging. */
int ht_batch_update_pinned_async(ht_batch *b, int32_t n_ctx, ht_ctx *const *ctxs, const int32_t *n_rows,
                                 const ht_row *const *rows);

/* Steps 4a-5 for several predicted contexts in one launch: as ht_force_async
 * per context, active ids from host arrays.  Results go to arrays the device
 * can write: device memory, or pinned host memory (hipHostMalloc), which the
 * host may read once the stream has been synchronised. */
int ht_batch_force_async(ht_batch *b, int32_t n_ctx, ht_ctx *const *ctxs, const int32_t *n_active,
                         const int32_t *const *active_ids, double *const *d_acc, double *const *d_jerk,
                         double *const *d_pot);

/* Device-resident steps for several contexts (each with ht_state_enable):
 * ht_batch_dev_next_block runs the scheduler of ht_dev_next_block for all of
 * them in one set of launches and returns t_next[k], n_active[k] and active[k]
 * (pinned, owned by ctxs[k]); ht_batch_dev_step then runs the force on all
 * those active sets in one launch (as ht_batch_force_async) and the corrector
 * for all of them in one more, with eta[k] and dt_tree[k] per context.  Same
 * results per context as its own ht_dev_next_block / ht_dev_step. */
int ht_batch_dev_next_block(ht_batch *b, int32_t n_ctx, ht_ctx *const *ctxs, double *t_next, int64_t *n_active,
                            const int32_t **active);
int ht_batch_dev_step(ht_batch *b, int32_t n_ctx, ht_ctx *const *ctxs, const double *eta, const double *dt_tree);

/* Batched device loop (Section 2, steps 2 and 4a-6 for many clusters): up
 * to engine_steps engine steps of the resident contexts ctxs[0..n_ctx-1],
 * queued on the batch's stream with no host round trip between them, in HIP
 * graphs of 32 engine steps.  In every engine step each context that is still
 * running takes one block step of its own: the scheduler of ht_dev_next_block,
 * the work plan of the device planner (the host planner's items, so each
 * context gets the bits of its own step-by-step run, alone or in any batch),
 * one force launch over all contexts' items and one corrector launch for all
 * of them.  Context k stops after its step at t_stop[k] (a tree time, where
 * the caller rebuilds it), before a block time beyond t_stop[k], or after
 * max_steps[k] steps, with eta[k] and dt_tree[k] as in ht_dev_step;
 * max_steps[k] = 0 makes it sit out the call: no kernel and no host code of
 * the call touches its state (it may be rebuilt meanwhile on another stream),
 * and t_last[k] is NaN.  The work runs on the batch's stream; the contexts
 * may live on other streams, and the caller makes sure that none of them has
 * work in flight there (the call waits only for its own stream).  Keeping
 * the same contexts from call to call (sitting out where needed) keeps the
 * captured graph.
 * Results: steps[k], t_last[k] (block time of its last step), particle_steps[k]
 * and pairs[k] (pair interactions summed) per context; step_ms (room for
 * engine_steps values) receives the wall time of every engine step in which
 * some context stepped, and *n_step_ms their number.  Synchronous (one wait,
 * at the end).  Needs fused prediction and whole-number gather costs;
 * engine_steps in [1, 4096].  The tables and the graph are kept while the
 * batch is called with the same contexts (same sizes and tunings).
 * HT_ERANGE if a plan exceeded a context's capacity or a step fell below
 * 2^-40: the steps before it stand. */
int ht_batch_dev_run(ht_batch *b, int32_t n_ctx, ht_ctx *const *ctxs, const double *eta, const double *dt_tree,
                     const double *t_stop, const int32_t *max_steps, int32_t engine_steps, int32_t *steps,
                     double *t_last, int64_t *particle_steps, int64_t *pairs, double *step_ms, int32_t *n_step_ms);

int ht_batch_sync(ht_batch *b);
int ht_batch_set_timing(ht_batch *b, int32_t enable);
int ht_batch_kernel_timing(ht_batch *b, double *force_ms, int64_t *launches, int64_t *pairs);
int ht_batch_last_stats(const ht_batch *b, int64_t *pairs, int32_t *work_items);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the direct
 * N^2 force of ht_force_direct_async, on caller-owned device arrays and with
 * no context, that calls no allocating routine.
 *
 * d_x, d_v [n][3] (FP64): predicted positions and velocities; d_m [n]: masses
 * (rounded to FP32 first in the mixed form, as the mixed j-records store
 * them); d_active [n_active]: particle indices in [0, n), in device memory,
 * so they cannot be checked before the launch: an index outside [0, n) gives
 * NaN in its output row.  d_acc, d_jerk [n_active][3], d_pot [n_active]:
 * outputs in active order.  precision: ht_precision (the pair arithmetic of
 * that form).  The j-range 0..n-1 is cut into j_splits equal ranges (1 to
 * 65535) summed by separate work-groups and then added in split order, so the
 * result's bits depend on j_splits only.  With j_splits > 1 the partial sums
 * go to one fixed device array of HT_NOALLOC_SCRATCH_BYTES per device, which
 * the library holds until the process ends; a call needing more
 * (j_splits * n_active * 56 bytes) fails with HT_ERANGE before any launch.
 * Every call on a device shares that array: calls that overlap in time on one
 * device (different streams, or threads) race and give wrong results.
 * Asynchronous on `stream` (a hipStream_t; NULL is the null stream) of
 * `device`, which must be the current device. */
#define HT_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int ht_force_direct_noalloc(int32_t device, void *stream, int32_t precision, int32_t n, const double *d_x,
                            const double *d_v, const double *d_m, double eps2, int32_t n_active,
                            const int32_t *d_active, int32_t j_splits, double *d_acc, double *d_jerk,
                            double *d_pot);

/* ---------------------------------------------------------------------------
 * Admission by device footprint (the served stream of cluster runs).  A pool
 * is a budget of device bytes on one GPU and the reservations held against
 * it; it allocates nothing itself.  ht_cluster_admit reserves what a cluster
 * with this configuration will hold: ht_workspace_bytes, plus ht_state_bytes
 * when resident (*bytes receives the figure).  HT_ENOMEM: it does not fit
 * beside the reservations held now (the caller waits for a release);
 * HT_ERANGE: it exceeds the whole budget and never fits (the caller refuses
 * it).  ht_pool_reserve holds other device memory against the budget (for
 * example a tree builder that clusters share, htd_device_bytes);
 * ht_pool_resize records a reservation's new size (a cluster moved to a
 * larger context, a builder that grew) and returns HT_ENOMEM when the pool is
 * then over its budget (the size is recorded either way).  Thread-safe. */
typedef struct ht_pool ht_pool;
int ht_pool_create(ht_pool **out, int32_t device, size_t budget_bytes);
int ht_pool_destroy(ht_pool *p);
int ht_cluster_admit(ht_pool *p, const ht_config *cfg, int32_t resident, int64_t *id, size_t *bytes);
int ht_pool_reserve(ht_pool *p, size_t bytes, int64_t *id);
int ht_pool_resize(ht_pool *p, int64_t id, size_t bytes);
int ht_cluster_release(ht_pool *p, int64_t id);
int ht_pool_usage(ht_pool *p, size_t *used, size_t *budget, int32_t *n_held);

/* Block until the context's queued work has finished. */
int ht_sync(ht_ctx *ctx);

/* Work-plan tuning.  The active particles of a group are covered by i-tiles
 * of T = 1, 2, 4, ..., 256 slots; a tile over a list of L entries is costed
 * rounds*(gather_cost+T) with rounds = ceil(L/256), a group gets the tiles of
 * least total cost, and tiles are split into list ranges only while the call
 * has fewer than about target_items items.  Defaults: 12, 2048.  Results
 * stay within the stated tolerances for any values (only the summation order
 * changes). */
int ht_set_tuning(ht_ctx *ctx, double gather_cost, double target_items);

/* Placement of a call's work items over the XCDs of the device (each with
 * its own L2; the paper's single pipeline array has no counterpart).  With
 * runs > 1 the host planner of the single-context list calls (ht_force,
 * ht_force_async, ht_step_async; not the direct sum) cuts the items, in
 * the order of their groups along the space-filling curve, into `runs`
 * stretches of equal modelled cost, orders each stretch longest first and
 * launches the force kernel so that work-group b takes the items of stretch
 * b % runs.  Work-groups go to the XCDs in turn, so with runs = the XCD count
 * each stretch runs on one XCD, whose L2 then serves the records that
 * neighbouring groups' lists share.  runs = 0: the device's XCD count; 1: off
 * (one longest-first order over all items).  Results do not depend on the
 * placement.  HT_EINVAL for runs outside [0, 16].  ht_get_placement returns
 * the runs in use and the device's XCD count. */
int ht_set_placement(ht_ctx *ctx, int32_t runs);
int ht_get_placement(const ht_ctx *ctx, int32_t *runs, int32_t *n_xcc);

/* Pair interactions the last force call summed (list entries x active
 * particles, self pairs included) and the number of work items it used. */
int ht_last_stats(const ht_ctx *ctx, int64_t *pairs, int32_t *work_items);

/* Timing of force-kernel launches: with timing enabled, every force launch
 * on this context's stream (batched launches count on their first context)
 * is bracketed by HIP events.  ht_kernel_timing synchronises the stream and
 * returns the summed kernel time in milliseconds, the number of launches and
 * the pair interactions they summed since timing was enabled or last read,
 * then starts a new tally. */
int ht_set_timing(ht_ctx *ctx, int32_t enable);
int ht_kernel_timing(ht_ctx *ctx, double *force_ms, int64_t *launches, int64_t *pairs);

/* Message for the last failure on the calling thread ("" if none). */
const char *ht_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HTREE_H */

/*
 * d2.h -- C ABI of the MI355X (gfx950) library for sparse-support
 * Wasserstein barycenters by the modified Bregman ADMM and the D2-clustering
 * loop built on them.
 *
 * Paper: Ye, Wu, Wang, Li, "Fast Discrete Distribution Clustering Using
 * Wasserstein Barycenter with Sparse Support" (IEEE TSP 2017).  Passages
 * are cited by section / equation label / algorithm name.
 *
 * Problem statement (Sec. 2): N instances P^(k) = {(w^(k)_j, x^(k)_j)},
 * j < m_k, with x^(k)_j in R^d and w^(k) in the simplex; K centroids
 * Q^(c) = {(w_i, x_i)}, i < m, one support size m for all centroids.
 *
 * Conventions for every call:
 *  - Host arrays are plain C arrays owned by the caller; the library copies
 *    what it keeps.  Host floating-point inputs/outputs are double; the
 *    device computes in the dtype chosen at d2_create.
 *  - Ragged instances use the paper's concatenated layout (Sec. 2, item 7):
 *    offsets[N+1] (int64, offsets[0] = 0, non-decreasing), instance k owns
 *    rows offsets[k] .. offsets[k+1]-1 of X (n x d, row-major) and W (n).
 *  - Plans (coupling matrices, Sec. 2 items 8-9) of instance k are m x m_k,
 *    column-major: entry (i, j) at m*offsets[k] + j*m + i of an m x n array.
 *  - Every call returns a d2_status; on error the outputs are untouched and
 *    d2_last_error() describes the failure.  No exception crosses the ABI.
 *  - A context is used by one host thread at a time.  All device work runs
 *    on the context's stream; calls that return host data synchronise it.
 *  - Library limits: 1 <= m <= 64, 1 <= m_k <= 64 with m_k * pad(m) <= 2048
 *    (pad(m) = next power of two >= max(m, 8)), d >= 1, K >= 1.
 */
#ifndef D2_H_
#define D2_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  D2_OK = 0,
  D2_EINVAL = 1,   /* bad argument or input data                          */
  D2_ENOMEM = 2,   /* device or host allocation failed                   */
  D2_EDEVICE = 3,  /* a HIP runtime call or kernel launch failed         */
  D2_ENUMERIC = 4, /* a non-finite value appeared in centroids or objective */
  D2_ESTATE = 5    /* call out of order (e.g. barycenter before labels)   */
} d2_status;

typedef enum { D2_F32 = 0, D2_F64 = 1 } d2_dtype;

typedef enum {
  D2_INIT_PRODUCT = 0, /* Pi2^0 = w_i w^(k)_j for every member (Sec. 5)     */
  D2_INIT_CACHED = 1,  /* cached Pi2 where the label did not change, else
                          the product (Sec. 5 warm start)                   */
  D2_INIT_LEARNED = 2  /* starting centroid proposed by the network attached
                          with d2_set_warm_start (gated against the current
                          centroid), Pi2^0 = product; not in the paper      */
} d2_init;

/* Parameters of one B-ADMM centroid update (Sec. 3.2, Algorithm "Centroid
 * Update with B-ADMM").  Defaults: rho0 2, tau 10, iters 100, eps 1e-16,
 * rule 1, xplan 0, init D2_INIT_CACHED.  rho = rho0 * mean cost of the
 * cluster at the call's initial support (Eq. (rho)); the support is updated
 * by Eq. (updatex) after every iteration n with (n+1) % tau == 0. */
typedef struct {
  double rho0;
  double eps;     /* added after each exponential product (Eq. badmmc0b/c1b) */
  int32_t tau;    /* support-update period; >= 1                           */
  int32_t iters;  /* B-ADMM iterations; >= 1                               */
  int32_t rule;   /* 1: R1, Eq. (badmmw); 2: R2, Eq. (badmmw2)             */
  int32_t xplan;  /* plan used by Eq. (updatex): 0 = Pi2 (only value)      */
  int32_t init;   /* d2_init                                               */
  int32_t fixed_support; /* 1: never update x (fixed-support barycenter)   */
} d2_badmm_params;

/* Parameters of the assignment distance: B-ADMM on one transport problem
 * with both marginals fixed (the updates of Sec. 3.2 without the weight
 * step), Pi2^0 = product coupling, rho = rho0 * mean cost of the pair. */
typedef struct {
  double rho0;
  double eps;
  int32_t iters;
  /* 1: skip a centroid whose lower bound sum_j w^(k)_j min_i C_ij (valid for
   * any plan with the instance's column sums, hence for Pi1) exceeds the
   * best distance found by more than 1e-4 relative; the labels and minimal
   * distances are those of the exhaustive search.  0: evaluate every pair. */
  int32_t prune;
} d2_ot_params;

typedef struct {
  int32_t iters;        /* iterations run                                 */
  int32_t n_empty;      /* clusters without members (centroid kept)       */
  int32_t launches;     /* kernel launches issued                         */
  int32_t graph;        /* 1 if the call replayed a captured HIP graph    */
  double ms;            /* device time of the call (HIP events)           */
} d2_badmm_stats;

typedef struct d2_ctx d2_ctx;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * to run on (NULL: the library creates its own default-priority stream).
 * dtype selects the device arithmetic (plans, costs, exponentials). */
d2_status d2_create(d2_ctx** out, int device, d2_dtype dtype, void* hip_stream);
/* Free every device buffer and graph of the context.  NULL is a no-op. */
void d2_destroy(d2_ctx* ctx);
/* Last error message of the context ("" if none). */
const char* d2_last_error(const d2_ctx* ctx);

/* Copy N ragged instances to the device (Sec. 2 notation).  Validates:
 * offsets[0] = 0 and non-decreasing, 1 <= m_k within the library limits,
 * finite X, W >= 0 and |sum_j w^(k)_j - 1| <= 1e-6 (each instance is then
 * renormalised in double).  Any earlier instances, labels and plans are
 * dropped.  Error D2_EINVAL names the first offending instance. */
d2_status d2_load_instances(d2_ctx* ctx, int64_t N, int32_t d,
                            const int64_t* offsets, const double* X,
                            const double* W);

/* Borrow N ragged instances that already sit in device memory (for
 * example PyTorch tensors), without copying.  offsets (host, N+1) as in
 * d2_load_instances.  dX is n x xs in the context's dtype (float for D2_F32,
 * double for D2_F64), xs = d rounded up to a multiple of 4, row-major, with
 * the padding columns t >= d equal to 0; dW is n weights in the same dtype.
 * Both must stay valid and unchanged until the context is destroyed or
 * loads other instances; the library never writes or frees them.  A device
 * check runs first (finite coordinates, zero padding, finite weights >= 0
 * summing to 1 within 1e-6 per instance, in double); on failure D2_EINVAL
 * names the first offending instance and the context is unchanged.  The
 * weights are used as given (no renormalisation). */
d2_status d2_load_instances_device(d2_ctx* ctx, int64_t N, int32_t d,
                                   const int64_t* offsets, const void* dX,
                                   const void* dW);

/* Load N instances over a symbolic support set (Sec. 5: the support
 * points are symbols of a finite set, e.g. amino acids or their n-grams,
 * with a given symbol-to-symbol dissimilarity; the support vectors are then
 * never updated).  offsets as in d2_load_instances; sym (n) holds each
 * support point's symbol in [0, S); W (n) the weights (checked and
 * renormalised as in d2_load_instances); D (S x S, row-major, finite,
 * >= 0, 1 <= S <= 16384) the cost of centroid symbol a against instance
 * symbol b at D[a * S + b] (it need not be symmetric).  All copied.  The
 * context then reports d = 1; its centroids are set with
 * d2_centroids_set_symbolic, d2_centroids_get returns each centroid
 * point's symbol (as a double) in Xc, and d2_barycenter updates the
 * weights only (the support step is skipped whatever fixed_support says).
 * Not available on such a context (D2_EINVAL): d2_centroids_set,
 * d2_centroids_init, d2_support_update, d2_objective_feasible, the
 * learned warm start. */
d2_status d2_load_instances_symbolic(d2_ctx* ctx, int64_t N,
                                     const int64_t* offsets,
                                     const int32_t* sym, const double* W,
                                     int32_t S, const double* D);

/* Centroids of a symbolic context: csym (K x m) are the support symbols of
 * each centroid, in [0, S); Wc (K x m) rows in the simplex as in
 * d2_centroids_set (whose plan-cache rule applies).  New symbols drop the
 * assignment's cross-round bounds. */
d2_status d2_centroids_set_symbolic(d2_ctx* ctx, int32_t K, int32_t m,
                                    const int32_t* csym, const double* Wc);

/* Set the K centroids: Xc is K x m x d, Wc is K x m (rows in the simplex,
 * |sum - 1| <= 1e-6, renormalised).  Requires loaded instances.  With K and
 * m unchanged the plan cache of the last d2_barycenter is kept, so that a
 * caller may continue a clustering run from centroids it adjusted; a caller
 * setting unrelated centroids passes D2_INIT_PRODUCT to the next
 * d2_barycenter.  d2_centroids_init and an accepted d2_ws_propose drop the
 * cache. */
d2_status d2_centroids_set(d2_ctx* ctx, int32_t K, int32_t m,
                           const double* Xc, const double* Wc);
/* Copy the centroids out (Xc: K x m x d, Wc: K x m). */
d2_status d2_centroids_get(d2_ctx* ctx, double* Xc, double* Wc);
/* Initialise centroid c from instance members[c] (Sec. 5): its support is
 * merged pairwise by Eq. (merge) -- the pair minimising
 * w_a w_b ||x_a - x_b||^2 / (w_a + w_b), ties to the smallest (a, b), the
 * merged point taking slot a -- until m points remain.  Each chosen member
 * needs m_k >= m.  The random choice of members is the caller's. */
d2_status d2_centroids_init(d2_ctx* ctx, int32_t K, int32_t m,
                            const int64_t* members);

/* Set / get the cluster label of every instance (values in [0, K)). */
d2_status d2_labels_set(d2_ctx* ctx, const int32_t* labels);
d2_status d2_labels_get(d2_ctx* ctx, int32_t* labels);

/* Assignment step (Algorithm "D2 Clustering"): l^(k) = argmin_c D(Q^(c),
 * P^(k)), D the B-ADMM transport value <C, Pi1> of `p`; ties go to the
 * lowest c.  Updates the context's labels (the previous labels are kept to
 * decide the warm start).  labels_out (N), dist_out (N, the minimal D) and
 * n_changed may be NULL. */
d2_status d2_assign(d2_ctx* ctx, const d2_ot_params* p, int32_t* labels_out,
                    double* dist_out, int64_t* n_changed);

/* Cross-round bounds of the pruned assignment (on = 1, the default).  The
 * pruning's lower bound LB(k, c) = sum_j w^(k)_j min_i C_ij depends on the
 * centroid only through its support points, so each pruned d2_assign
 * stores a lower bound on sqrt(LB) for every (instance, centroid) pair
 * (N x K floats on the device) and the next one lowers it by the largest
 * distance any support point of the centroid moved in between (the
 * triangle inequality, as in the paper's Sec. 5 use of Elkan's method):
 * pairs whose decayed bound already clears the best distance skip their
 * cost block.  Labels and minimal distances stay those of the exhaustive
 * search.  on = 0 frees the bounds; if they cannot be allocated the
 * assignment prunes within the round only. */
d2_status d2_set_assign_bounds(d2_ctx* ctx, int32_t on);

/* Pair counts of the last d2_assign: pairs run through the transport
 * iterations, pairs whose m x m_k cost block was formed (those passing the
 * cheap bound of the pruning; every pair without pruning) and the total
 * number of (instance, centroid) pairs.  Any pointer may be NULL. */
d2_status d2_assign_pairs(const d2_ctx* ctx, int64_t* evaluated,
                          int64_t* costed, int64_t* total);

/* Centroid update (Sec. 3.2, Algorithm "Centroid Update with B-ADMM") for
 * all K clusters of the current labels in one batched pass: Lambda = 0,
 * Pi2^0 per p->init, `iters` iterations of Eq. (badmmc0b)-(badmmc1),
 * R1/R2 and Eq. (badmm2), support updates every tau.  Empty clusters keep
 * their centroid.  The final Pi2 is cached for the next call's warm start.
 * stats may be NULL. */
d2_status d2_barycenter(d2_ctx* ctx, const d2_badmm_params* p,
                        d2_badmm_stats* stats);

/* Eq. (updatex) for every non-empty cluster from the cached Pi2 plans:
 * x_i = sum_k sum_j Pi2_ij x^(k)_j / sum_k sum_j Pi2_ij.  Requires a
 * previous d2_barycenter on the current labels. */
d2_status d2_support_update(d2_ctx* ctx);

/* Per-round record passed to the d2_cluster callback. */
typedef struct {
  int32_t round;
  int64_t n_changed;     /* labels changed by this round's assignment      */
  double assign_obj;     /* mean over instances of the minimal D           */
  double ms_assign;      /* device time of the assignment                  */
  double ms_barycenter;  /* device time of the centroid update             */
} d2_round_info;

typedef void (*d2_round_cb)(const d2_round_info* info, void* user);

/* D2-clustering (Algorithm "D2 Clustering") for `rounds` rounds from the
 * current centroids: assignment, then d2_barycenter with the cached-plan
 * warm start (Sec. 5).  cb may be NULL. */
d2_status d2_cluster(d2_ctx* ctx, int32_t rounds, const d2_badmm_params* bp,
                     const d2_ot_params* op, d2_round_cb cb, void* user);

/* Multi-modal instances (Sec. 5: an instance is an array of distributions,
 * e.g. a protein's amino-acid and tripeptide histograms).  Modality i of
 * every instance lives in context ctxs[i] (its own supports, d, m, m_k,
 * vector or symbolic); all contexts are on one device with the same N and
 * K, and instance k of each is the same object.  The assignment distance
 * of (instance, centroid) is the sum over modalities of the B-ADMM
 * transport values of `p`; labels = argmin, ties to the lowest centroid.
 * Every pair of every modality is evaluated (no pruning); the per-pair
 * distances are summed in modality order in an N x K double buffer of
 * ctxs[0].  The labels (and the minimal summed distances) are written to
 * every context; labels_out (N), dist_out (N) and n_changed (against the
 * previous labels of ctxs[0]) may be NULL.  Errors are reported through
 * ctxs[0]. */
d2_status d2_assign_multi(int32_t n_modal, d2_ctx* const* ctxs,
                          const d2_ot_params* p, int32_t* labels_out,
                          double* dist_out, int64_t* n_changed);

/* D2-clustering of multi-modal instances: `rounds` rounds of
 * d2_assign_multi followed by d2_barycenter on every modality's context
 * (the modalities' centroids are updated separately, Sec. 5; product start
 * in a first round without a plan cache, else bp->init).  The callback
 * gets the summed barycenter time of the modalities. */
d2_status d2_cluster_multi(int32_t n_modal, d2_ctx* const* ctxs,
                           int32_t rounds, const d2_badmm_params* bp,
                           const d2_ot_params* op, d2_round_cb cb,
                           void* user);

/* Parameters of the subgradient-descent centroid update (Appendix A,
 * Algorithm "Centroid Update with Subgradient Descent").  Defaults: alpha
 * 0.5, zeta 1, tau 10, iters 20, fixed_support 0, max_pivots 0. */
typedef struct {
  double alpha;          /* Eq. (stepsize): step length in log-weights    */
  double zeta;           /* Eq. (stepsize): cap on alpha / ||gradient||   */
  int32_t tau;           /* support update every tau iterations (>= 1)    */
  int32_t iters;         /* iterations (>= 1)                             */
  int32_t fixed_support; /* 1: never update the support                   */
  int32_t max_pivots;    /* per transport LP; 0: 50 (m + max m_k)         */
} d2_sg_params;

typedef struct {
  int32_t iters;     /* iterations run                                     */
  int32_t lp_failed; /* transport LPs stopped by the pivot cap (summed)    */
  int64_t pivots;    /* simplex pivots over all LPs                        */
  int32_t launches;  /* kernel launches                                    */
  int32_t pad;
  double ms;         /* device time (HIP events)                           */
} d2_sg_stats;

/* Subgradient-descent centroid update for all K clusters of the current
 * labels (Appendix A; the refinement the paper compares B-ADMM with, here
 * usable from B-ADMM's centroids).  Every iteration n: the support update
 * Eq. (updatex) from the previous iteration's plans when n > 0 and
 * n % tau == 0 (never for symbolic supports or fixed_support = 1); for
 * every instance the exact transport LP Eq. (primal) against its cluster's
 * centroid (network simplex in FP64 on the device, one wavefront per
 * instance) giving its plan and the duals of the row constraints; per
 * cluster the mean over members of the duals minus their mean (Eq.
 * (dualvar)), the gradient of the objective in s with w = softmax(s), the
 * step Eq. (stepsize) sigma = min(alpha / ||grad_s||, zeta), s -= sigma
 * grad_s, s -= mean(s), w = softmax(s).  At the start s = log w -
 * mean(log w).  d2_objective then returns per iteration the exact
 * objective (1/N_c) sum_k W^2 at that iteration's centroid (before its
 * step); the last plans become the plan cache (Pi2 = Pi1 = the LP plans).
 * An LP stopped by the pivot cap keeps its current basis (counted in
 * stats->lp_failed).  stats may be NULL. */
d2_status d2_subgradient(d2_ctx* ctx, const d2_sg_params* p,
                         d2_sg_stats* stats);

/* Hold rho at the given per-cluster values (K, finite, > 0) in the
 * following d2_barycenter calls instead of Eq. (rho) (rho0 times the mean
 * cost at the call's initial support; rho is the method's one
 * hyper-parameter).  NULL returns to Eq. (rho).  New centroids of another
 * K or m drop the values.  d2_objective reports the rho used. */
d2_status d2_set_rho(d2_ctx* ctx, const double* rho);

/* Objective trace of the last d2_barycenter: trace[n*K + c] =
 * (1/N_c) sum_k <C^(k), Pi1^(k)> of iteration n (0 for empty clusters);
 * `max_iters` bounds the rows written.  rho (K, may be NULL) gets each
 * cluster's rho. */
d2_status d2_objective(d2_ctx* ctx, double* trace, int32_t max_iters,
                       double* rho);

/* Primal residual trace of the last d2_barycenter: residual[n*K + c] =
 * (1/N_c) sum_k sum_ij |Pi1^(k)_ij - Pi2^(k)_ij| after iteration n, the
 * violation of the splitting constraint Pi1 = Pi2 whose multiplier
 * Eq. (badmm2) updates (0 for empty clusters); `max_iters` bounds the rows
 * written. */
d2_status d2_residual(d2_ctx* ctx, double* residual, int32_t max_iters);

/* Plans of instance k after the last d2_barycenter, each m x m_k
 * column-major (Pi1, Pi2, Lambda); any pointer may be NULL. */
d2_status d2_plans_get(d2_ctx* ctx, int64_t k, double* P1, double* P2,
                       double* L);

/* Per-kernel timing.  With profiling on, every kernel launch of the
 * context is bracketed by two HIP events recorded on the context's stream,
 * and the elapsed times are accumulated per kernel kind when the call that
 * launched them synchronises.  Kinds: "rho_cost", "init_a", "iter_ba",
 * "b_final", "xnum_only", "assign", "finalize".  One "iter_ba" unit is one
 * B-ADMM iteration: the launches of all slot buckets (d2_set_bucketing)
 * inside one event pair. */
typedef struct {
  char name[24];
  int64_t launches;
  double total_ms;
} d2_kernel_stat;

d2_status d2_set_profiling(d2_ctx* ctx, int32_t on);
/* Copy up to `cap` accumulated records (kinds with at least one launch) and
 * their number; `reset` != 0 clears the accumulators afterwards. */
d2_status d2_kernel_stats(d2_ctx* ctx, d2_kernel_stat* out, int32_t cap,
                          int32_t* count, int32_t reset);

/* Capture the launch sequence of d2_barycenter in a HIP graph on first use
 * (per iterations / tau / rule / schedule / sizes) and replay it (on = 1,
 * the default), or issue every launch from the host (on = 0).  With
 * profiling on, launches are issued from the host so that each can be
 * bracketed by events. */
d2_status d2_set_graph(d2_ctx* ctx, int32_t on);

/* Cache policy of the plan state (Pi1, Lambda, cost cache) in the
 * per-iteration kernel of FP32 contexts: 0 automatic (the default:
 * non-temporal accesses when that state exceeds the 256 MiB last-level
 * cache, else the default policy), 1 default policy, 2 non-temporal.
 * Results do not depend on it (bitwise). */
d2_status d2_set_cache_policy(d2_ctx* ctx, int32_t policy);

/* Launch schedule of the barycenter kernels: instances per workgroup chunk
 * (1 .. 4096) and wavefronts per workgroup (1, 2 or 4).  Results do not
 * depend on the schedule beyond floating-point summation order.  The
 * autotuner (paper_1510_00012_amd.autotune) picks these per workload. */
d2_status d2_set_schedule(d2_ctx* ctx, int32_t chunk_instances,
                          int32_t waves_per_group);

/* Slot buckets of the per-iteration plan-update kernel.  An instance's
 * tile needs ceil(m_k / (64 / pad(m))) register slots per lane; instances
 * are grouped by the power of two above that count, and each group runs as
 * its own launch of a kernel specialised for it (fewer registers, more
 * wavefronts in flight for small instances).  A group holding fewer than
 * min_pct % of the plan entries joins the next larger group; 100 gives one
 * launch for all instances (the default: on the measured workloads the
 * extra launches cost more than the higher occupancy gains), 0 one launch
 * per group present.
 * Results depend on it only through floating-point summation order. */
d2_status d2_set_bucketing(d2_ctx* ctx, int32_t min_pct);

/* Autotuner: times d2_barycenter (`iters` iterations, product start) on the
 * current labels for each candidate schedule -- instances per chunk in
 * {16, 32, 64, 128, 256} x wavefronts per workgroup in {2, 4} x slot
 * bucketing threshold in {100, 10} (d2_set_bucketing) -- keeps the fastest
 * (set on the context) and reports it.  Centroids are restored afterwards;
 * any warm-start plan cache is dropped, so call it before the first
 * centroid update.  Any output pointer may be NULL; ms_best gets the best
 * device time. */
d2_status d2_autotune(d2_ctx* ctx, const d2_badmm_params* p,
                      int32_t* chunk_out, int32_t* waves_out,
                      int32_t* bucket_out, double* ms_best);

/* Round-boundary checkpoint of a clustering run (Sec. 5 keeps each
 * member's Pi2 across rounds for the warm start; this saves exactly what
 * the next round reads): the centroids, the labels, the cache labels and
 * the cached Pi2 plans, and the launch schedule (results depend on it
 * through summation order), with a fingerprint of the loaded instances and
 * a checksum.  Written to path + ".tmp" and renamed, so a crash never
 * leaves a half-written checkpoint under `path`.  The assignment's
 * cross-round bounds are not saved (they only skip work).  D2_ESTATE
 * without instances and centroids. */
d2_status d2_checkpoint_save(d2_ctx* ctx, const char* path);
/* Restore a checkpoint into a context holding the same instances (same N,
 * n, d, dtype and fingerprint).  The file is read and checked in full
 * before anything changes: a missing, truncated, corrupt or foreign file
 * gives D2_EINVAL and leaves the context as it was.  Continuing the run
 * afterwards gives bitwise the results of the uninterrupted run. */
d2_status d2_checkpoint_load(d2_ctx* ctx, const char* path);

/* Achievable-bandwidth probe (not part of the paper: the reference point
 * beside the published HBM peak for the plan-update roofline).  Copies a
 * buffer of `bytes` (>= 1 MiB; rounded down to 16 bytes) to a second one on
 * `device` with a plain vectorised kernel, reps + 1 times; the fastest of
 * the last reps launches gives *gbs = 2 * bytes / time (read + write, in
 * GB/s) and *ms its duration (may be NULL).  Allocates and frees its two
 * buffers; D2_ENOMEM if they do not fit. */
d2_status d2_copy_probe(int device, int64_t bytes, int32_t reps, double* gbs,
                        double* ms);

/* Assignment step that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Computes what d2_assign computes on a
 * fresh context (no previous labels, no cross-round bounds): labels[k] =
 * argmin_c of the B-ADMM transport value of `p` between centroid c and
 * instance k, ties to the lowest c, dist[k] its minimal value.
 * Everything is the caller's device memory on `device`:
 *   offsets  N+1 int64 (offsets[0] = 0, 1 <= m_k <= mk_max),
 *   X        n x xs values of `dtype` (float / double), xs = d rounded up
 *            to a multiple of 4, padding columns 0, row-major,
 *   W        n instance weights of `dtype` (each instance in the simplex),
 *   Xc, Wc   K x m x d and K x m doubles (Wc rows are divided by their sum),
 *   labels   N int32 (out), dist N doubles (out).
 * The per-centroid data the kernels need besides these live in a fixed
 * 8 MiB device array of the library, one per GPU, held until the process
 * ends: K x pad(m) x (d + 1) doubles plus K x (pad(m) x xs + d + 1) values
 * of `dtype` (256-byte aligned parts) must fit in it, else D2_EINVAL with
 * the sizes in `err`.  The call only enqueues work on hip_stream (NULL: the
 * device's null stream) and returns without waiting; the outputs are
 * valid once the stream reaches that point.  Calls that overlap on one GPU
 * (other streams, other host threads) share the array and race; calls on
 * one stream are ordered.  Argument errors (D2_EINVAL, checked before any
 * device call) and launch failures (D2_EDEVICE) write a message to err
 * (err_len bytes with the terminating zero; err may be NULL).  The device
 * data is not inspected: an instance with m_k < 1 or m_k > mk_max gets
 * label -1 and a NaN distance; offsets outside X and W are undefined.
 * N = 0 returns D2_OK without touching the device. */
d2_status d2_assign_noalloc(int32_t device, void* hip_stream, d2_dtype dtype,
                            int64_t N, int32_t d, int32_t mk_max,
                            const int64_t* offsets, const void* X,
                            const void* W, int32_t K, int32_t m,
                            const double* Xc, const double* Wc,
                            const d2_ot_params* p, int32_t* labels,
                            double* dist, char* err, int32_t err_len);

/* Sizes: N, n, d, K, m of the context (any pointer may be NULL). */
d2_status d2_sizes(const d2_ctx* ctx, int64_t* N, int64_t* n, int32_t* d,
                   int32_t* K, int32_t* m);

/* Barycenter objective of the current centroids under the plans of the last
 * d2_barycenter (Eq. (badmm_prob) evaluated at a feasible point): every
 * instance's Pi1 is rounded to a coupling whose row sums are the centroid
 * weights and whose column sums are w^(k) exactly (rows scaled down to at
 * most w_c, then columns to at most w^(k), then the rank-one correction
 * err_r err_c^T / |err_r|_1), and its cost under C(x) is taken in FP64.
 * Each value is an upper bound on W^2 between the centroid and the
 * instance, so per_cluster[c] = (1/N_c) sum_{k in c} value_k bounds the
 * cluster's objective from above.  per_instance (N) and per_cluster (K,
 * 0 for empty clusters) may be NULL.  The per-cluster means are summed on
 * the host in instance order.  D2_ESTATE if the labels changed since the
 * last d2_barycenter. */
d2_status d2_objective_feasible(d2_ctx* ctx, double* per_instance,
                                double* per_cluster);

/* ---- Learned warm start ------------------------------------------------
 * Not part of the paper: a deep-sets network proposes each cluster's
 * initial centroid for the centroid update of Sec. 3.2 from the cluster's
 * members.  For the points y_j of member k (weights w_j, m_k points) of a
 * cluster with weighted mean mu and RMS radius s:
 *   f = [(y_j - mu)/s, m_k w_j] (zero padded to din = roundup(d+1, 16)),
 *   h = relu(relu(f W1 + b1) W2 + b2),  g = sum_j (w_j / N_c) h,
 *   o = relu(relu(g V1 + e1) V2 + e2) V3 + e3  (outp = roundup(m(d+1), 32)),
 *   x_i = mu + s o[i d .. i d + d),  w = softmax(o[m d .. m d + m)).
 * Matrix products take BF16 operands with FP32 accumulation (MFMA); the
 * master parameters are FP32, one flat vector ordered W1 (din x H), b1,
 * W2 (H x H), b2, V1 (H x H), e1, V2 (H x H), e2, V3 (H x outp), e3, each
 * matrix row-major with the input index first.
 * Training loss per cluster with targets (x*, w*), in standardised
 * coordinates t_j = (x*_j - mu)/s, nn by first minimum:
 *   sum_j w*_j |D_nn(j) - t_j|^2 + sum_i w_i |D_i - t_nn(i)|^2
 *   - sum_i q_i log w_i,   q_i = sum of w*_j with nn(j) = i;
 * the batch loss is the mean over the batch's clusters.
 * Limits: m <= 64, d <= 64, m d <= 2048, H in {32, 64, 96, 128}.  A handle
 * lives on one device and serves any context on that device whose m and d
 * match; its calls run on the context's stream. */
typedef struct d2_ws d2_ws;

typedef struct {
  double lr;     /* Adam step size                              */
  double beta1;  /* first-moment decay                          */
  double beta2;  /* second-moment decay                         */
  double eps;    /* denominator guard                           */
  double clip;   /* global gradient-norm clip (0: no clipping)  */
} d2_ws_opt;

/* Number of parameters for (m, d, hidden), or -1 outside the limits. */
int64_t d2_ws_param_count(int32_t m, int32_t d, int32_t hidden);

/* Create a network on `device` with initial parameters theta (host,
 * d2_ws_param_count values, copied).  Adam state starts at zero. */
d2_status d2_ws_create(d2_ws** out, int32_t device, int32_t m, int32_t d,
                       int32_t hidden, const float* theta);
void d2_ws_destroy(d2_ws* ws);
const char* d2_ws_last_error(const d2_ws* ws);

/* Copy parameters in (resets the Adam state) / out (host buffers). */
d2_status d2_ws_params_set(d2_ws* ws, const float* theta);
d2_status d2_ws_params_get(d2_ws* ws, float* theta);

/* Take the context's current K centroids as the training targets of its
 * clusters (cluster c of later batches is trained toward centroid c). */
d2_status d2_ws_targets_from(d2_ws* ws, d2_ctx* ctx);

/* Mean loss (may be NULL) and its gradient (host, param_count values, may
 * be NULL) over the batch clusters[0..nb) of the context's current labels.
 * Every listed cluster must be non-empty; D2_ESTATE without targets or if
 * the context's K changed since d2_ws_targets_from. */
d2_status d2_ws_grad(d2_ws* ws, d2_ctx* ctx, const int32_t* clusters,
                     int32_t nb, double* loss, float* grad);

/* One Adam step (bias-corrected, after global-norm clipping) on the batch's
 * gradient; loss (may be NULL) gets the batch loss before the step. */
d2_status d2_ws_train_step(d2_ws* ws, d2_ctx* ctx, const int32_t* clusters,
                           int32_t nb, const d2_ws_opt* opt, double* loss);

/* Save / load the network: parameters, Adam moments and step count (so
 * that training resumes exactly), with its shape (m, d, hidden) and a
 * checksum.  Load requires a handle of the same shape; on any error
 * (missing, truncated, foreign or corrupt file) D2_EINVAL and the handle is
 * unchanged.  Save writes path + ".tmp" and renames it. */
d2_status d2_ws_save(d2_ws* ws, const char* path);
d2_status d2_ws_load(d2_ws* ws, const char* path);

/* Attach a network for D2_INIT_LEARNED calls of d2_barycenter (NULL
 * detaches).  gate 0: the proposal replaces every finite centroid; gate 1:
 * the product-coupling bound of d2_ws_propose decides; gate >= 2: a probe
 * decides -- B-ADMM runs `gate` iterations (product start) from the
 * current centroid and from the proposal, and per cluster the start whose
 * rounded-plan objective (d2_objective_feasible) is lower afterwards is
 * kept (ties keep the current centroid); the call then starts from the
 * kept centroids.  The caller keeps the handle alive while it is
 * attached. */
d2_status d2_set_warm_start(d2_ctx* ctx, d2_ws* ws, int32_t gate);

/* Propose a centroid for every non-empty cluster of the context's current
 * labels.  The product-coupling bound sum_k sum_ij w_i w_j^(k) C_ij of the
 * proposal is compared with that of the context's current centroid (the
 * plain initial centroid); the proposal replaces it iff it is finite and,
 * when gate != 0, its bound is not larger.  accepted[c] (K) gets 1 / 0, or
 * -1 for empty clusters; bound_prop and bound_plain (K) the two bounds (NaN
 * for empty clusters); any of the three may be NULL. */
d2_status d2_ws_propose(d2_ws* ws, d2_ctx* ctx, int32_t gate,
                        int32_t* accepted, double* bound_prop,
                        double* bound_plain);

#ifdef __cplusplus
}
#endif
#endif /* D2_H_ */

/*
 * ccmi.h - C ABI of libccmi, proximal-distance convex clustering on MI355X.
 *
 * The method (Chen, Chi, Ranola, Lange, "Convex Clustering: An Attractive
 * Alternative to Hierarchical Clustering"):
 *   minimise f_mu(U) = 1/2 sum_{(i,f) observed} (x_if - u_if)^2
 *                      + mu sum_{i<j} w_ij ||u_i - u_j||          (eq_lindsten,
 *                                                          eq_missing_analog)
 * by the proximal-distance MM algorithm of Section "The Proximal Distance
 * Algorithm": split v_ij = u_i - u_j (eq_proxdist), smooth the distance to the
 * constraint set by eps (dist_eps), majorise twice (first_surrogate,
 * sqrt_root_majorization, second_surrogate), and iterate
 *   projection (A, D A) = P_C(U, V)         block-descent projection
 *   d = sqrt(||U - A||^2 + ||V - D A||^2 + eps)
 *   v_e <- max(1 - mu w_e d / (rho ||b_e||), 0) b_e,  b = D A     (V update)
 *   u_i <- (d y_i + rho a_i) / (d + rho), y = x observed, u elsewhere
 *                                                   (U update, Missing Data)
 * The projection is approximated by one Jacobi sweep of the paper's block
 * update per MM iteration, started from the previous projection; the fixed
 * points are those of the exact projection.
 *
 * Conventions
 *   - Every function returns a cc_status and never throws.  On an error
 *     cc_last_error_message() (thread-local) describes it.
 *   - "device" pointers are HIP device memory on the current device; "host"
 *     pointers are ordinary host memory.
 *   - Matrices are row-major, one row per case (point), with a leading
 *     dimension in elements (ldx >= p).  This is the same byte layout as the
 *     paper's p x n column-major X with cases as columns.
 *   - Edges are unordered pairs {i, j} with positive weight, given once as
 *     (ei[e], ej[e]) with 0 <= ei[e] < ej[e] < n, 0-based, no duplicates
 *     (Methods: E is the set of pairs with w_ij > 0).
 *   - Work is enqueued on the stream given at creation (a hipStream_t passed
 *     as void*, NULL = the null stream).  Functions that return results to
 *     host memory synchronise that stream; results written to device memory
 *     are ordered on the stream and the caller synchronises.
 *   - A cc_problem_t is used by one host thread at a time.  Distinct problems
 *     may run concurrently on distinct streams.
 *   - Arguments are validated on the host before anything is launched; on
 *     CC_ERR_INVALID_ARG nothing has been written.
 */
#ifndef CCMI_H
#define CCMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cc_status;
enum {
  CC_OK = 0,
  CC_ERR_INVALID_ARG = 1,   /* bad argument; nothing was written            */
  CC_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed             */
  CC_ERR_HIP = 3,           /* a HIP runtime call failed                    */
  CC_ERR_NUMERIC = 4,       /* d or the objective became non-finite         */
  CC_ERR_STATE = 5          /* call not valid in the problem's state        */
};

/* Element type of caller-supplied data matrices. */
enum { CC_DTYPE_F32 = 0, CC_DTYPE_F64 = 1 };

/* Storage precision of the solver state.
 *   CC_PREC_F32   U, A and the pair sweep in FP32; reductions FP64.
 *   CC_PREC_MIXED U in FP64; A as the FP32 copy of A that the pair sweep
 *                 gathers (which runs in FP32) plus an FP32 low half, 48
 *                 significant bits; the point arithmetic, reductions, d, the
 *                 objective, the convergence test and every fusion decision
 *                 in FP64.  Default.
 *   CC_PREC_F64   everything FP64. */
enum { CC_PREC_F32 = 0, CC_PREC_MIXED = 1, CC_PREC_F64 = 2 };

typedef struct cc_problem *cc_problem_t;
typedef struct cc_batch *cc_batch_t;
typedef struct cc_server *cc_server_t;

/* Solver options.  Fill with cc_default_opts() and then change fields.
 *   eta         accuracy knob: eps = (eta * rho)^2 when eps <= 0.  The MM
 *               fixed point lies O(eta) from the exact minimiser of f_mu.
 *   rho         penalty constant of the proximal-distance method ("rho bigger
 *               than a Lipschitz constant"); <= 0 selects
 *               rho = 2 sqrt(||M o (X - xbar)||^2 + mu^2 sum_e w_e^2), a bound
 *               on the multiplier norm at the optimum.  Recomputed per mu.
 *   eps         smoothing constant of dist_eps; <= 0 selects (eta rho)^2.
 *   tol         stop after MM iteration m >= 2, taken when m+1 is a
 *               multiple of test_every = K, if
 *                 sqrt(||U_{m+1}-U_{m+1-K}||^2 + ||A_m - A_{m-K}||^2) / K
 *                    <= tol * eta * max(1, ||U_{m+1}||_F)
 *               with eta = sqrt(eps)/rho; 0 disables the test.  The paper
 *               leaves the stopping rule open; the window K averages out
 *               rounding-level jitter of reduced-precision state.
 *   max_iter    MM iteration cap per mu (not an error when reached).
 *   check_every iterations enqueued between host checks of the stop flag.
 *   warm_start  1: start from the problem's current state (the previous
 *               solve's final state, or an imported one); 0: start from the
 *               initial state U = A = X-tilde, V = D X-tilde.
 *   record_objective  1: keep the objective of every iteration
 *               (cc_get_trace).
 *   test_every  the window K of the stopping test, >= 1 (default 64).
 *   proj_sweeps Jacobi sweeps of the paper's block update per MM iteration
 *               (block-descent projection: the u_i are updated until they
 *               stabilise), 1..64, each started from the previous sweep and
 *               the first from the previous projection A'; default 1.  Any
 *               count has the fixed points of the exact projection; more
 *               sweeps bring each iteration's projection closer to it.
 *               Batched and served solves take 1. */
typedef struct {
  int32_t struct_size; /* sizeof(cc_solve_opts) */
  double eta;          /* default 1e-2 */
  double rho;          /* default 0 (auto) */
  double eps;          /* default 0 (auto) */
  double tol;          /* default 1e-6 */
  int32_t max_iter;    /* default 200000 */
  int32_t check_every; /* default 256 */
  int32_t warm_start;  /* default 1 */
  int32_t record_objective; /* default 0 */
  int32_t test_every;  /* default 64 */
  int32_t proj_sweeps; /* default 1 */
} cc_solve_opts;

/* Result of one solve (one mu).  objective and d belong to the last MM
 * iteration performed; rel_change is the quantity compared in the stopping
 * test divided by max(1, ||U||_F). */
typedef struct {
  int32_t iters;      /* MM iterations performed */
  int32_t converged;  /* 1 if the stopping test passed */
  int32_t n_clusters; /* connected components of the fused edges */
  int32_t status;     /* cc_status of this solve */
  double gamma;       /* mu */
  double objective;   /* F = loss + mu sum w ||v|| + rho d */
  double d;           /* smoothed distance d of the last iteration */
  double rel_change;
  double rho;
  double eps;
  double seconds;     /* wall time of the solve, host clock */
} cc_solve_info;

const char *cc_status_string(cc_status s);
const char *cc_last_error_message(void);
void cc_default_opts(cc_solve_opts *opts);
/* Library version as major*10000 + minor*100 + patch. */
int32_t cc_version(void);

/* ---------------------------------------------------------------------
 * Problem lifetime
 * ---------------------------------------------------------------------
 * cc_problem_create: copy a clustering problem into library-owned device
 * memory and set the initial state.
 *   n, p        cases and predictors, both >= 1.
 *   x_dtype     CC_DTYPE_F32 or CC_DTYPE_F64 for X.
 *   X           device, n rows of ldx elements; only observed entries are
 *               read (missing ones may hold anything, NaN included).
 *   mask        device uint8, n rows of ldm bytes, nonzero = observed
 *               (the index set Gamma of eq_missing_analog); NULL = all
 *               observed.
 *   n_edges     |E| >= 0.  ei, ej: device int32 endpoint arrays; w: device
 *               float64 weights, finite and > 0 (eq_weighting, or any prior
 *               weights).
 *   precision   CC_PREC_* for the solver state.
 *   stream      hipStream_t for all work of this problem.
 * The inputs are copied; the function synchronises the stream before
 * returning, so the caller may free them afterwards.  Observed X must be
 * finite.  out must not be NULL; on success *out owns the device state until
 * cc_problem_destroy, on failure *out is NULL. */
cc_status cc_problem_create(int64_t n, int64_t p, int32_t x_dtype,
                            const void *X, int64_t ldx, const uint8_t *mask,
                            int64_t ldm, int64_t n_edges, const int32_t *ei,
                            const int32_t *ej, const double *w,
                            int32_t precision, void *stream,
                            cc_problem_t *out);
cc_status cc_problem_destroy(cc_problem_t prob);
/* Dimensions (host outputs, any may be NULL). */
cc_status cc_problem_dims(cc_problem_t prob, int64_t *n, int64_t *p,
                          int64_t *n_edges, int32_t *precision);

/* ---------------------------------------------------------------------
 * Solving
 * ---------------------------------------------------------------------
 * cc_solve: run the MM iteration of Section "The Proximal Distance
 * Algorithm" (projection, smoothed distance d, V update, U update with the
 * missing-data majorisation of Section "Missing Data") at mu = gamma >= 0
 * until the stopping test passes or max_iter iterations are done.  opts may
 * be NULL (defaults).  info (host, may be NULL) is filled synchronously.
 * Afterwards the state holds U, the factored V and the fusion pattern of the
 * final iterate.  Returns CC_ERR_NUMERIC if d or the objective became
 * non-finite (an ordinary status: the kernels run to their end); the state
 * is then invalid, and the next warm-started solve starts from the initial
 * state (cc_reset_state and cc_set_state restore one explicitly).  Argument
 * errors (CC_ERR_INVALID_ARG) leave the state untouched. */
cc_status cc_solve(cc_problem_t prob, double gamma, const cc_solve_opts *opts,
                   cc_solve_info *info);

/* cc_solve_path: the solution path over the regularisation parameter
 * (Section "Evaluation of Clusters": one set of centres per mu, clusters
 * read off as mu grows).  Solves gammas[0..n_gamma-1] (host) in the given
 * order, each warm-started from the previous one's final state (the first one
 * from the current state if opts->warm_start, else from the initial state).
 * labels (device int32, n_gamma*n, may be NULL): row g holds the cluster
 * label of every case after gammas[g], the smallest case index of its
 * cluster.  U_path (device float32, n_gamma rows of n*p, row-major with
 * leading dimension p, may be NULL): the centres after each gamma.
 * infos (host, n_gamma entries, may be NULL).  Every gamma must be finite
 * and >= 0: all are checked before the first is solved (CC_ERR_INVALID_ARG,
 * state untouched).  Stops at the first gamma whose solve fails and returns
 * its status (infos up to it are filled). */
cc_status cc_solve_path(cc_problem_t prob, int32_t n_gamma,
                        const double *gammas, const cc_solve_opts *opts,
                        int32_t *labels, float *U_path, cc_solve_info *infos);

/* ---------------------------------------------------------------------
 * Results
 * --------------------------------------------------------------------- */
/* Centres U of the current state (the last MM iterate U_{m+1}; the
 * minimiser of f_mu is approximated O(eta) closely, Section "The Proximal
 * Distance Algorithm") into device memory of out_dtype, n rows of ldu
 * elements.  Asynchronous on the problem's stream. */
cc_status cc_get_U(cc_problem_t prob, int32_t out_dtype, void *U, int64_t ldu);
/* Cluster labels (device int32, n): connected components of the fused edges
 * (v_e = 0 after the last V update: the group soft-threshold of the V
 * update sets v_e exactly to zero when ||b_e|| <= mu w_e d / rho, and the
 * paper reads clusters off the centres that have merged), each labelled by
 * its smallest case index.  n_clusters (host, may be NULL) receives the
 * count and makes the call synchronous. */
cc_status cc_get_labels(cc_problem_t prob, int32_t *labels,
                        int32_t *n_clusters);
/* Fused flag per input edge, in input order (device uint8, n_edges): 1 when
 * the V update's shrinkage set v_e to zero (fusion of the centres of its two
 * cases), else 0.  Asynchronous on the problem's stream. */
cc_status cc_get_fused_edges(cc_problem_t prob, uint8_t *fused);
/* Objective of every iteration of the last solve with record_objective = 1
 * (host float64, up to cap values); *count receives the number stored. */
cc_status cc_get_trace(cc_problem_t prob, double *F, int64_t cap,
                       int64_t *count);

/* ---------------------------------------------------------------------
 * Kernel timing
 * ---------------------------------------------------------------------
 * cc_profile: sample_every > 0 brackets the two stages of every
 * sample_every-th MM iteration with HIP events on the problem's stream and
 * accumulates their durations; 0 turns sampling off.  Enabling clears the
 * statistics.  cc_kernel_stats (host outputs, 2 entries each: the point
 * sweep, which begins by finishing the previous iteration, then the edge
 * stage) returns the mean duration in milliseconds and the number of
 * sampled launches. */
cc_status cc_profile(cc_problem_t prob, int32_t sample_every);
cc_status cc_kernel_stats(cc_problem_t prob, double *avg_ms, int64_t *launches);

/* ---------------------------------------------------------------------
 * State checkpoint (warm starts across processes or problems)
 * ---------------------------------------------------------------------
 * The state of the MM iteration is (U, V) (Section "The Proximal Distance
 * Algorithm"); V is kept factored as V = diag(s) D A', A' the projection it
 * was shrunk from, so the state is (U, s, A').  Warm starts along the path
 * (Section "Evaluation of Clusters") carry it from one mu to the next; a
 * checkpoint carries it across processes.  cc_state_size gives the
 * byte size of the serialised state; export writes it to host memory,
 * import reads it back into a problem of the same n, p, edge set and
 * precision (CC_ERR_INVALID_ARG otherwise).  cc_reset_state returns to the
 * initial state. */
cc_status cc_state_size(cc_problem_t prob, size_t *bytes);
cc_status cc_export_state(cc_problem_t prob, void *buf, size_t bytes);
cc_status cc_import_state(cc_problem_t prob, const void *buf, size_t bytes);
cc_status cc_reset_state(cc_problem_t prob);
/* Set the state from device arrays: U and A' (float64, n rows of ld) and s
 * (float64, n_edges, in input edge order, each in [0, 1]).  The values are
 * rounded to the precision's storage: FP32 (CC_PREC_F32), FP64 U and A' as
 * an FP32 high half plus an FP32 low half, 48 significant bits
 * (CC_PREC_MIXED), FP64 (CC_PREC_F64). */
cc_status cc_set_state(cc_problem_t prob, const double *U, const double *A,
                       int64_t ld, const double *s);
/* Read the state into device arrays of the same form. */
cc_status cc_get_state(cc_problem_t prob, double *U, double *A, int64_t ld,
                       double *s);

/* ---------------------------------------------------------------------
 * Weights and input preparation
 * ---------------------------------------------------------------------
 * cc_build_knn_weights: the weights of eq_weighting,
 *   w_ij = 1{i ~_k j} exp(-phi d_ij^2),  d_ij = ||x_i - x_j||,
 * where i ~_k j when j is among the k nearest neighbours of i or i among
 * those of j (self excluded, distance ties to the lower index).  Distances
 * use the matrix with missing entries replaced by observed column means.
 * Candidates are ranked with a Gram matrix product on the matrix cores and
 * then re-ranked with exact FP64 distances.  The result is exact: a row is
 * accepted only when its k-th FP64 distance lies below the smallest FP32
 * distance left out minus a bound on that distance's rounding error;
 * otherwise the row is ranked again over 8x more candidates (at least 512),
 * then over all rows (n <= 12289).  CC_ERR_NUMERIC when a row still cannot
 * be certified (only above that n, for rows with more than 12288 others
 * within FP32 rounding of their k-th neighbour).
 *   k           1 <= k < n.
 *   phi         >= 0 literal; < 0 means |phi| / median(d^2 over the edge
 *               set), the lower median.
 *   normalize   1: scale the weights to sum to 1 over the edge set (the
 *               paper's normalisation, equivalent to rescaling mu).
 *   ei, ej, w   device outputs with room for capacity edges (n*k always
 *               suffices); edges come out sorted by (ei, ej), ei < ej.
 *   n_edges     host output, |E|.  phi_used: host output, may be NULL.
 * Supports n <= 16384. */
cc_status cc_build_knn_weights(int64_t n, int64_t p, int32_t x_dtype,
                               const void *X, int64_t ldx,
                               const uint8_t *mask, int64_t ldm, int32_t k,
                               double phi, int32_t normalize, int32_t *ei,
                               int32_t *ej, double *w, int64_t capacity,
                               int64_t *n_edges, double *phi_used,
                               void *stream);

/* cc_standardize_columns: in place on device X (x_dtype, n rows of ldx),
 * each column to mean 0 and variance 1 over its observed entries
 * (divisor = observed count); a constant column becomes 0; missing entries
 * are left untouched.  The paper advises this when predictors have widely
 * different scales (Methods, after eq_lindsten). */
cc_status cc_standardize_columns(int64_t n, int64_t p, int32_t x_dtype,
                                 void *X, int64_t ldx, const uint8_t *mask,
                                 int64_t ldm, void *stream);

/* cc_standardize_columns_noalloc: for callers that cannot allocate device
 * memory (code between the allocation points of a serving loop, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * cc_standardize_columns, but the column statistics live in a fixed device
 * array of the library instead of memory allocated per call: it calls no
 * hipMalloc or hipFree.  Each GPU the library runs on holds 1 MiB of it
 * until the process ends.  Takes p <= 65536 (CC_ERR_INVALID_ARG beyond,
 * nothing written).  Every call on a GPU uses that GPU's one array, so calls
 * that overlap on one GPU (from several host threads or on unordered
 * streams) race; calls ordered on one stream, or separated by a
 * synchronisation, do not.  Like cc_standardize_columns it synchronises the
 * stream (it reads back the count of non-finite observed entries). */
cc_status cc_standardize_columns_noalloc(int64_t n, int64_t p, int32_t x_dtype,
                                         void *X, int64_t ldx,
                                         const uint8_t *mask, int64_t ldm,
                                         void *stream);

/* cc_components: connected components of the subgraph of edges with
 * keep[e] != 0 (device uint8, may be NULL = all), labels (device int32, n)
 * = smallest index in each component; n_components host output. */
cc_status cc_components(int64_t n, int64_t n_edges, const int32_t *ei,
                        const int32_t *ej, const uint8_t *keep,
                        int32_t *labels, int32_t *n_components, void *stream);

/* ---------------------------------------------------------------------
 * Batched solves
 * ---------------------------------------------------------------------
 * Many independent problems, each along its own gamma path (Methods: the
 * solution path over the regularisation parameter, with warm starts), run
 * in the same launches: per MM iteration one point-sweep and one edge-sweep
 * launch cover every instance, and each instance keeps its own rho, eps, d,
 * objective and stopping test, and moves to its next gamma on the device.
 *
 * cc_batch_create: problems[0..n_inst-1] (host array of handles, distinct,
 * same precision, p <= 1024); n_gamma (host, n_inst
 * entries >= 1) and gammas (host, the paths one after another, each value
 * finite and >= 0).  opts may be NULL (defaults); each gamma is solved as
 * cc_solve would with these options, warm-started from the previous one
 * (the first from the problem's current state).  autotune != 0 times a few
 * iterations of each point-sweep tile width (64, 128, 256 features) with
 * about 1, 4 and 16 work items per wave (a wave with several prefetches the
 * next), and keeps the fastest; it leaves every problem at its initial
 * state.  The batched edge sweep takes 4 work items per wave whatever that
 * choice.  The
 * batch refers to the problems (it does not own them): destroy the batch
 * first.  A problem's solver state belongs to the batch while it runs.
 *
 * cc_batch_run: runs every path to its end and waits for it.  labels
 * (device int32, may be NULL): for each instance in order, n_gamma[b] rows
 * of n_b labels as cc_solve_path writes them.  infos (host, sum of n_gamma
 * entries, may be NULL): per (instance, gamma) as cc_solve fills them, with
 * seconds = time from the start of the run to the end of that gamma.
 * latency_ms (host, n_inst entries, may be NULL): time from the start of
 * the run to the end of each instance's path.  Afterwards each problem's
 * state is the final state of its path (cc_get_U etc. read it).
 * Returns CC_ERR_NUMERIC if any instance's d or objective became
 * non-finite (its path stops there; the others finish).
 *
 * cc_batch_config (host outputs, any may be NULL), for the instance with
 * the most work: its point-sweep features per lane (vec: tile width
 * 64 * vec) and work items per wave; the MM iterations per graph replay;
 * and tune_us (9 entries): the autotuner's microseconds per batched
 * iteration when that instance's class took (vec, items per wave) = (1,1),
 * (1,4), (1,16), (2,1), (2,4), (2,16), (4,1), (4,4), (4,16) (zeros without
 * autotuning).
 *
 * cc_batch_tuning: the autotuner's choice per class of instances.  The
 * autotuner groups instances by the width of their rows (class 0: p <= 64,
 * 1: <= 128, 2: <= 256, 3: wider) and by the point-sweep work items at the
 * width's natural tile (0: <= 512, 1: <= 2048, 2: more), and gives each
 * class its own point-sweep launch, timing the 9 candidates above for one
 * class at a time (classes with more work first, the others keeping their
 * choice).  Host outputs: *n_classes (may be NULL) the number of classes;
 * for the first cap classes, classes[5 c + 0..4] = width class, size class,
 * instances, vec, items per wave, and us[c] (may be NULL) the microseconds
 * per batched iteration with the choices; inst_class (n_inst entries, may
 * be NULL) the class of each instance.  Without autotuning there are no
 * classes (instance classes -1) and every instance takes vec from its row
 * width (p <= 64: 1, <= 128: 2, else 4) and one item per wave. */
cc_status cc_batch_create(int32_t n_inst, const cc_problem_t *problems,
                          const int32_t *n_gamma, const double *gammas,
                          const cc_solve_opts *opts, int32_t autotune,
                          cc_batch_t *out);
cc_status cc_batch_run(cc_batch_t batch, int32_t *labels, cc_solve_info *infos,
                       double *latency_ms);
cc_status cc_batch_config(cc_batch_t batch, int32_t *vec, int32_t *items_per_wave,
                          int32_t *graph_iters, double *tune_us);
cc_status cc_batch_tuning(cc_batch_t batch, int32_t cap, int32_t *n_classes,
                          int32_t *classes, double *us, int32_t *inst_class);
cc_status cc_batch_destroy(cc_batch_t batch);

/* ---------------------------------------------------------------------
 * Served solves (continuous batching)
 * ---------------------------------------------------------------------
 * Requests (a data matrix, its kNN weight parameters and a gamma path)
 * queue on the host and are admitted first come, first served while the
 * device bytes of the admitted requests stay within hbm_budget (a request
 * is admitted alone whatever its size).  Admission builds the weights
 * (cc_build_knn_weights) and the problem on the device; every admitted
 * request then shares the launches of the others, as in a batch, and
 * leaves them when its path is done; requests arriving meanwhile join at
 * the next round.  Each path is solved as cc_solve_path would solve it.
 *
 * cc_server_create: precision CC_PREC_*; opts may be NULL (defaults);
 * max_active (1..4096) admitted requests at most; round_iters (even, >= 2)
 * MM iterations per cc_server_step; all work on stream.
 * cc_server_submit: host inputs, copied: X (float32, n rows of p, p <=
 * 1024, 2 <= n <= 16384), mask (uint8, 1 = observed, may be NULL), k and
 * phi as for cc_build_knn_weights, gammas (n_gamma >= 1 values).  *ticket
 * identifies the request.
 * cc_server_step: admits what the budget allows, then runs one round over
 * the admitted requests and waits for it.  Host outputs (may be NULL): the
 * admitted and waiting counts after the round and the number of requests
 * that finished in it.
 * cc_server_status: state (CC_REQ_*) and times in seconds since the server
 * was created: submitted, admitted, done (host clock; done is the end of
 * the round that finished the path).
 * cc_server_result: for a CC_REQ_DONE request, labels (device int32,
 * n_gamma rows of n, may be NULL), infos (host, n_gamma, may be NULL;
 * seconds = admission to done) as cc_solve_path gives them, and U (device
 * float32, n rows of p, may be NULL): the centres at the end of the path.
 * cc_server_release: frees a request that is not running (its budget share
 * returns).  cc_server_memory (host outputs, may be NULL): the device bytes
 * counted against the budget by the admitted and finished requests not yet
 * released, and the budget.  A request whose admission failed (state
 * CC_REQ_FAILED, its status from cc_server_result) holds no device memory
 * and is not counted.  cc_server_destroy frees every request. */
#define CC_REQ_WAITING 0
#define CC_REQ_ACTIVE 1
#define CC_REQ_DONE 2
#define CC_REQ_FAILED 3
cc_status cc_server_create(int32_t precision, const cc_solve_opts *opts,
                           int64_t hbm_budget, int32_t max_active,
                           int32_t round_iters, void *stream, cc_server_t *out);
cc_status cc_server_submit(cc_server_t server, int64_t n, int64_t p,
                           const float *X, const uint8_t *mask, int32_t k,
                           double phi, int32_t n_gamma, const double *gammas,
                           int64_t *ticket);
cc_status cc_server_step(cc_server_t server, int32_t *n_active,
                         int32_t *n_waiting, int32_t *n_done);
cc_status cc_server_status(cc_server_t server, int64_t ticket, int32_t *state,
                           double *t_submit, double *t_admit, double *t_done);
cc_status cc_server_result(cc_server_t server, int64_t ticket, int32_t *labels,
                           cc_solve_info *infos, float *U);
cc_status cc_server_release(cc_server_t server, int64_t ticket);
cc_status cc_server_memory(cc_server_t server, int64_t *used, int64_t *budget);
cc_status cc_server_destroy(cc_server_t server);

/* ---------------------------------------------------------------------
 * Extras the paper suggests around the solver
 * ---------------------------------------------------------------------
 * cc_pca: principal components of the original data, for viewing the
 * cluster path on them (Evaluation of Clusters).  X (device, x_dtype, n
 * rows of ldx) and mask (device, may be NULL) as for cc_problem_create;
 * missing entries are replaced by their observed column means and the
 * columns centred by those means.  Returns the top r right singular vectors
 * of the centred matrix, V (device FP64, p x r row-major: V[f * r + c]),
 * each signed so that its entry of largest magnitude is positive; the
 * singular values sval (host FP64, r, decreasing); center (device FP64, p,
 * may be NULL) the column means.  Subspace iteration with r + 8 columns for
 * iters steps (0 = 100), then a Rayleigh-Ritz step; the accuracy of column
 * c improves as (sigma_{r+9} / sigma_c)^(2 iters).  1 <= r <= min(16, n, p).
 *
 * cc_solve_path_pc: cc_solve_path, except that instead of U the path
 * returns its projection on the device (Discussion: project before any
 * transfer): proj (device FP64, n_gamma x n x r), proj[g][i][c] =
 * sum_f (u_if - center_f) V[f][c] for the U reported at gamma g.  V (device
 * FP64, p x r as cc_pca writes it), center (device FP64, p, may be NULL =
 * zero), 1 <= r <= 16.  labels and infos as for cc_solve_path.
 *
 * cc_min_connected_k: the smallest k <= k_max for which the kNN graph of
 * cc_build_knn_weights (same neighbours, ties and imputation) is connected,
 * found by bisection over k with a connected-components search per step
 * (Results, "Impact of the Constants k and phi"); -1 when it is not
 * connected at k_max.  n_components: components at k_max (host output).
 * 1 <= k_max < n, k_max <= 1024, n <= 16384.
 *
 * cc_composite_weights: weights w_e = exp(-phi d_e^2) over given edges
 * (device ei, ej, n_edges) from the composite distance of eq
 * composite_distance, d_ij = alpha ||x_i - x_j|| + (1 - alpha) dist(y_i, y_j)
 * with X (device, x_dtype, n rows of ldx, p columns; p may be 0) and mask
 * (device, may be NULL: missing entries take their observed column mean, as
 * for cc_build_knn_weights) and coordinates Y (device FP64, n rows of ldy,
 * q <= 8 columns).  dist is Euclidean over the coordinates, a coordinate
 * with period[t] > 0 (host, q entries, may be NULL) taken modulo that period
 * (the shorter way round); geodesic != 0 needs q = 2 and takes (latitude,
 * longitude) in degrees, dist = radius (<= 0 means 1) times the
 * great-circle angle.  phi, normalize and phi_used as for
 * cc_build_knn_weights; w: device output, n_edges.  The result goes to
 * cc_problem_create as the edge weights. */
cc_status cc_pca(int64_t n, int64_t p, int32_t x_dtype, const void *X, int64_t ldx,
                 const uint8_t *mask, int64_t ldm, int32_t r, int32_t iters,
                 double *V, double *sval, double *center, void *stream);
cc_status cc_solve_path_pc(cc_problem_t prob, int32_t n_gamma, const double *gammas,
                           const cc_solve_opts *opts, int32_t *labels, int32_t r,
                           const double *V, const double *center, double *proj,
                           cc_solve_info *infos);
cc_status cc_min_connected_k(int64_t n, int64_t p, int32_t x_dtype, const void *X,
                             int64_t ldx, const uint8_t *mask, int64_t ldm,
                             int32_t k_max, int32_t *k_min, int32_t *n_components,
                             void *stream);
cc_status cc_composite_weights(int64_t n, int64_t n_edges, const int32_t *ei,
                               const int32_t *ej, int64_t p, int32_t x_dtype,
                               const void *X, int64_t ldx, const uint8_t *mask,
                               int64_t ldm, int32_t q,
                               const double *Y, int64_t ldy, const double *period,
                               int32_t geodesic, double radius, double alpha,
                               double phi, int32_t normalize, double *w,
                               double *phi_used, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CCMI_H */

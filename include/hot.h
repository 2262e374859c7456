/*
 * hot.h -- C ABI of libhot, an MI355X (gfx950) implementation of HOT, the
 * Halpern accelerating method for optimal transport between two histograms
 * on an m x n grid with squared Euclidean ground cost (arXiv 2408.00598).
 *
 * The library solves the reduced OT model (Sec. 2.1, eq. partite-graph /
 * standLP) with Algorithm 2 (alg:HOT), the linear-time solve of Prop. 3
 * (prop:linsol_OT) and the relative KKT stopping rule (eq. kkt_res), and
 * recovers a transport plan with Algorithm 1 (alg:transportplan).
 *
 * Conventions shared by every entry point
 *  - Histograms are caller-owned DEVICE buffers of m*n doubles, row-major:
 *    mu[i*n + j] is the mass of bin (i, j).  They must be nonnegative,
 *    finite, and have equal totals (the paper assumes total 1, Sec. 2.1).
 *  - Flow and dual vectors exported by hot_solution_export use the paper's
 *    vectorisation (def:A1A2A3): x = [f1; f2] with f1_{i,k,j} at
 *    (j*m + k)*m + i and f2_{k,j,l} at m*m*n + (l*n + j)*m + k; y = [y1; y2;
 *    y3] with y1 at j*m+k, y2 at m*n + j*m+i, y3 at 2*m*n + l*m+k (the row
 *    (l,k) = (n-1, m-1) is removed, def:A4), 3*m*n - 1 entries in total.
 *  - Every function returns a status; nothing aborts or throws across the
 *    ABI.  On error, output buffers are left unspecified unless stated.
 *  - Streams: work is enqueued on the given hipStream_t (0 = null stream).
 *    Synchronous calls (hot_solve, hot_recover_plan) return when done.
 *  - One context may be used by one host thread at a time (an internal mutex
 *    serialises concurrent calls on the same context).
 */
#ifndef HOT_H
#define HOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hot_stream_t; /* same type as hipStream_t */

typedef enum {
  HOT_OK = 0,
  HOT_E_INVALID = 1,       /* bad argument or histogram (see hot_problem) */
  HOT_E_NOMEM = 2,         /* device allocation failed / budget exceeded */
  HOT_E_DEVICE = 3,        /* HIP runtime error */
  HOT_E_NOT_CONVERGED = 4, /* max_iter reached; result holds the last iterate */
  HOT_E_BUSY = 5,          /* server full or handle still running */
  HOT_E_CANCELLED = 6,
  HOT_E_NUMERIC = 7        /* non-finite value appeared in the iteration */
} hot_status;

typedef enum {
  HOT_FP64 = 0,        /* flow state stored and streamed in FP64 */
  HOT_FP32_STREAM = 1  /* flow state stored in FP32; all reductions, the
                          linear solve and per-element arithmetic in FP64 */
} hot_precision;

/* hot_problem.flags */
#define HOT_FLAG_RESTART 0x1u     /* restart rule on (the default reading) */
#define HOT_FLAG_FIXED_ITERS 0x2u /* run exactly max_iter updates of Alg. 2,
                                     no stopping test, no restart; the result
                                     is w_bar at the final iterate */
#define HOT_FLAG_ADMM 0x4u        /* generalized ADMM baseline of Sec. 4.1:
                                     Step 4 of Alg. 2 replaced by
                                     w <- (1 - rho) w + rho w_bar with
                                     rho = hot_problem.relax; no restarts */
#define HOT_FLAG_ABS_KKT 0x8u     /* stop when ||R(w_bar)|| <= tol, R the
                                     residual map stated before Prop.
                                     complexity, instead of eq. kkt_res */
#define HOT_FLAG_SIGMA_UPDATE 0x10u /* with the restart rule: at every restart
                                     set sigma <- ||x_bar - X|| / ||A^T (y_bar - Y)||,
                                     (X, Y) the w_bar of the previous restart
                                     (0 before the first); the paper leaves
                                     sigma open (Algorithm 2 only asks
                                     sigma > 0).  Costs one more state-sized
                                     buffer and one more stream on check and
                                     restart passes. */
#define HOT_FLAG_ESCALATE 0x20u   /* with HOT_FP32_STREAM: when the relative KKT
                                     stops improving above tol (not halved
                                     over the last max(1000, k_best / 4)
                                     iterations, at least two restarts
                                     done), widen the state to FP64 in place
                                     (exactly), start a new epoch there (one
                                     restart pass, counted in restarts and
                                     iters) and continue with FP64 streams;
                                     hot_result.escalated_at records the
                                     iteration.  hot_solve and the server
                                     act on it; batches and hot_solve_noalloc
                                     ignore it. */

typedef struct {
  int32_t m, n;            /* grid rows, columns: 1 <= m, n <= 1024 */
  const double *mu1;       /* device, m*n, source histogram */
  const double *mu2;       /* device, m*n, target histogram */
  double tol;              /* relative KKT tolerance (eq. kkt_res), > 0 */
  int32_t max_iter;        /* iteration cap (>= 1) */
  int32_t check_every;     /* KKT/restart check cadence T (>= 1; 10 typical) */
  double sigma;            /* penalty sigma of Alg. 2; <= 0 selects ||b||/||c|| */
  int32_t prec;            /* hot_precision */
  uint32_t flags;          /* HOT_FLAG_* */
  double relax;            /* rho of HOT_FLAG_ADMM, in (0, 2); <= 0 selects
                              1.7 (the experiments' value); ignored otherwise */
  const double *coord_row; /* device, m finite positions u_i of the grid rows,
                              or NULL for u_i = i */
  const double *coord_col; /* device, n finite positions v_j of the grid
                              columns, or NULL for v_j = j.  Bin (i,j) sits at
                              (u_i, v_j) and the ground cost is the squared
                              distance (u_i-u_k)^2 + (v_j-v_l)^2: the
                              non-uniform bins of the color-transfer
                              application (Sec. 4.2); A and b are unchanged,
                              only c (eq. def:c) follows the positions.
                              Positions need not be sorted or distinct. */
} hot_problem;

typedef struct {
  double primal_obj;  /* <c, x_bar>: the reduced objective, = W2^2 at optimum */
  double dual_obj;    /* <b, y_bar> */
  double kkt;         /* max(res_primal, res_dual, res_comp), eq. kkt_res */
  double res_primal;  /* ||A x_bar - b|| / (1 + ||b||) */
  double res_dual;    /* ||A^T y_bar + z_bar - c|| / (1 + ||c||) */
  double res_comp;    /* ||min(x_bar, z_bar)|| / (1 + ||x_bar|| + ||z_bar||) */
  double sigma;       /* sigma used */
  double seconds;     /* wall time of the solve on the host clock */
  double kkt_abs;     /* ||R(w_bar)|| = sqrt(||b - A x_bar||^2 +
                         ||min(x_bar, z_bar)||^2 + ||c - A^T y_bar - z_bar||^2) */
  int32_t iters;      /* updates performed (Alg. 2 iterations) */
  int32_t restarts;
  int32_t status;     /* hot_status of this problem */
  int32_t escalated_at; /* HOT_FLAG_ESCALATE: iteration count at which the
                           FP32 streams were widened to FP64, 0 if never */
  double feaserr;     /* max(||min(x_bar, 0)|| / (1 + ||x_bar||), res_primal): the
                         relative primal feasibility error of the experiments
                         (Sec. 4.1, the metric feaserr) */
} hot_result;

typedef struct hot_ctx hot_ctx;
typedef struct hot_solution hot_solution;
typedef struct hot_batch hot_batch;
typedef struct hot_server hot_server;

/* Create a context on HIP device `device`.  Owns the workspace pool.
 * Returns HOT_E_DEVICE if the device cannot be used (e.g. no GPU).
 * Launch-shape defaults can be overridden through environment variables read
 * here (integers; for measurement and tuning, none changes a result beyond
 * summation order): HOT_ITEM_ELEMS (flow elements per slab-pass workgroup),
 * HOT_MIN_ITEMS, HOT_UNROLL (1 or 2 rows per wave step), HOT_VPL_TARGET
 * (16-byte vectors per lane per row), HOT_NT_STORE (0/1), HOT_PINGPONG (0/1),
 * HOT_SMALL_SIDE (largest slab side of the wave-per-slab pass, 0 = none),
 * HOT_FUSE (0: separate plain and check/restart slab kernels),
 * HOT_ROW_GROUP (slabs per solve wave; results unchanged), HOT_REDUCE_GROUP
 * (row slots per reduce workgroup; results unchanged), HOT_BATCH_GROUPS (1..4
 * concurrent groups of a batch), HOT_SOLVE_PRE (1, the default / 0: the solve
 * issues its decision-free loads before / after the decision; results
 * unchanged).
 * HOT_NO_GRAPH=1 launches every iteration directly instead of through
 * captured graphs.  HOT_TEST_NAN_AFTER=q (failure-path tests only) makes
 * hot_solve write a NaN into the flow state between graph launch q and q+1,
 * so that the solve must end with HOT_E_NUMERIC. */
hot_status hot_ctx_create(int device, hot_ctx **out);
void hot_ctx_destroy(hot_ctx *ctx);

/* Text of the last error recorded on ctx (never NULL; "" if none). */
const char *hot_ctx_last_error(const hot_ctx *ctx);
const char *hot_status_string(hot_status s);

/* Measurement.  With profiling on, solves launch the iteration kernels
 * directly (no graphs) and time every slab pass with a hipEvent pair on the
 * solver's stream.  hot_ctx_profile_read fills out[4] with counters summed
 * over all solves since profiling was last switched:
 *   out[0] slab-pass launches timed, out[1] their total seconds (events),
 *   out[2] algorithmic bytes streamed by the timed slab passes (state read +
 *          anchor read when separate + state write, padding excluded),
 *   out[3] iterations launched. */
hot_status hot_ctx_set_profiling(hot_ctx *ctx, int on);
hot_status hot_ctx_profile_read(hot_ctx *ctx, double *out);

/* Autotuner of the slab-pass launch shape.  For the shapes and precision of
 * probs (histogram values are ignored: uniform histograms are solved),
 * times `iters` fixed iterations (slab pass, reduce and solve, in captured
 * graphs, host wall clock around the run after the set-up has finished),
 * each pass streaming the state, a (zero)
 * Halpern anchor and the new state as every pass after the first restart
 * does, under each candidate workgroup size (2^11 ..
 * 2^17 flow elements per workgroup), row unroll (1, 2) and 16-byte vectors
 * per lane per slab row (2, 4), and keeps the fastest in ctx for launches of the
 * same precision, size class (floor(log2) of the total flow elements) and
 * pair-count class (floor(log2) of the number of problems).  cache_path
 * (nullable): the choice is appended as a JSON line keyed by device
 * architecture, precision, size class and pair-count class;
 * hot_autotune_load reads such a file (later lines win, entries of other
 * architectures are ignored).  out (nullable, 5 doubles): chosen
 * elements per workgroup, chosen unroll, its seconds per iteration, the
 * built-in rule's, chosen vectors per lane.  The chunking changes the
 * summation order of column partial sums, so tuned results can differ from
 * untuned ones by rounding. */
hot_status hot_autotune(hot_ctx *ctx, const hot_problem *probs, int32_t count,
                        int32_t iters, const char *cache_path, double *out);
hot_status hot_autotune_load(hot_ctx *ctx, const char *cache_path);

/* Device bytes one problem needs (state buffers, sums, dual vectors), laid
 * out with the built-in launch-shape rule.  Pure host arithmetic; 0 for
 * invalid sizes. */
size_t hot_footprint_bytes(int32_t m, int32_t n, int32_t prec, uint32_t flags);
/* The same with the context's launch-shape tuning (environment overrides and
 * loaded autotuner choices), which is what hot_solve allocates and what the
 * server admits by. */
size_t hot_ctx_footprint_bytes(hot_ctx *ctx, int32_t m, int32_t n, int32_t prec,
                               uint32_t flags);

/* Upper bound on the number of plan entries hot_recover_plan may write:
 * m*n*(m+n-1) from Algorithm 1 plus 2*m*n - 1 from the marginal repair. */
int64_t hot_plan_capacity(int32_t m, int32_t n);

/* Solve one problem with Algorithm 2 (Steps 1-4, restart rule when
 * HOT_FLAG_RESTART is set) until the relative KKT residual of w_bar is
 * <= tol at a check, or max_iter.  Blocks until done.
 * sol_out (nullable): receives a handle that keeps the final iterate on the
 * device for hot_recover_plan / hot_solution_export; free it with
 * hot_solution_free.  res (required) receives the result.
 * Returns HOT_OK, HOT_E_NOT_CONVERGED (res filled with the last iterate),
 * HOT_E_NUMERIC, HOT_E_INVALID (bad sizes, tol, negative/non-finite mass or
 * totals differing by more than 1e-9 relative), HOT_E_NOMEM, HOT_E_DEVICE. */
hot_status hot_solve(hot_ctx *ctx, const hot_problem *prob, hot_stream_t stream,
                     hot_solution **sol_out, hot_result *res);

/* Copy the final iterate of a solution into caller-owned DEVICE buffers in
 * the paper's ordering (any pointer may be NULL to skip it):
 * xbar, zbar: N = m*m*n + m*n*n doubles; ybar: 3*m*n - 1 doubles;
 * s: the Halpern state x/sigma + z of the last update, N doubles. */
hot_status hot_solution_export(hot_ctx *ctx, const hot_solution *sol,
                               hot_stream_t stream, double *xbar, double *ybar,
                               double *zbar, double *s);
void hot_solution_free(hot_solution *sol);

/* The Halpern anchor of the final epoch (Algorithm 2, Step 4: the point w^0
 * the epoch's updates are pulled toward, here the state s^0 = x^0/sigma + z^0
 * the epoch restarted from, or 0 before the first restart) in the paper's
 * ordering, into a caller-owned DEVICE buffer of N doubles (nullable), and
 * (host, nullable, 4 doubles) the control values the solve ended with:
 * info[0] the epoch counter k of the last update, info[1] the Halpern weight
 * 1/(k+2) of the next update (1 - rho/2 for the ADMM baseline), info[2]
 * sigma, info[3] 0 if the anchor is zero, 1 if it is the state itself (ADMM
 * baseline, first update after a restart), 2 if it is a buffer of its own. */
hot_status hot_solution_anchor(hot_ctx *ctx, const hot_solution *sol,
                               hot_stream_t stream, double *s0, double *info);

/* hot_solve without any allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Every device buffer of the solve is carved from one static
 * device array of hot_noalloc_capacity() bytes (64 MiB) that each device
 * holds until the process ends: a problem whose workspace does not fit
 * (with the built-in launch rule, square grids above 136 x 136 with FP32
 * streams or 110 x 110 in FP64) is rejected with HOT_E_INVALID and a
 * message giving the bytes it needs.  The iteration runs
 * on `stream` by direct launches (no graph, no event, no pinned buffer); the
 * call returns when done.  Same kernels, launch shapes and order as
 * hot_solve, so `res` and the iterate are bit-identical to it (res->seconds
 * aside).  xbar (N doubles), ybar (3*m*n - 1 doubles): nullable caller-owned
 * DEVICE buffers receiving the final x_bar and y_bar in the paper's ordering.
 * The array keeps the last call's contents (what must start at zero is
 * cleared by each call).  Calls on one context are serialised by its mutex;
 * calls through different contexts on the same device share the array and
 * race if they overlap, so such callers must serialise them. */
hot_status hot_solve_noalloc(hot_ctx *ctx, const hot_problem *prob, hot_stream_t stream,
                             double *xbar, double *ybar, hot_result *res);
size_t hot_noalloc_capacity(void);

/* Algorithm 1 on the clipped flows max(x_bar, 0) of `sol`, followed by the
 * marginal repair (rows above mu1 scaled down, then columns above mu2, then
 * the remaining deficits coupled north-west-corner in bin order).  Writes
 * entries (src bin i*n+j, dst bin k*n+l, mass) to caller-owned DEVICE arrays
 * of `capacity` entries; capacity >= hot_plan_capacity(m, n) is required
 * (HOT_E_INVALID otherwise).  *nnz receives the entry count.  marg_err
 * (host, 4 doubles, nullable): L1 errors of row and column marginals before
 * repair, then after repair.  Entries of bin (k,j) are contiguous, ordered
 * by (k*n + j), then by source row i, then by target column l; the repair
 * entries follow.  Scratch (about 16 bytes per flow element) comes from a
 * buffer the context keeps at the largest size a recovery has needed, until
 * hot_ctx_destroy; recoveries on one context run one at a time. */
hot_status hot_recover_plan(hot_ctx *ctx, const hot_solution *sol,
                            hot_stream_t stream, int32_t *src, int32_t *dst,
                            double *mass, int64_t capacity, int64_t *nnz,
                            double *marg_err);

/* Solve A A^T y = R with the structured solve of Prop. 3 on the device.
 * R, y: DEVICE buffers of 3*m*n - 1 doubles in the paper's row order. */
hot_status hot_aat_solve(hot_ctx *ctx, int32_t m, int32_t n, const double *R,
                         double *y, hot_stream_t stream);

/* Batched solves: many problems (sizes may differ) share every launch; the
 * iteration loop runs device-side in captured HIP graphs.  The batch is
 * split into a few groups balanced by flow elements (two by default), each
 * with its own stream and graph, iterated concurrently so that one group's
 * latency-bound reduce and solve kernels overlap another's streaming slab
 * pass; with profiling on, the batch runs as one group.  Submit returns
 * once the work is enqueued and a host thread drives it; hot_batch_wait
 * blocks, fills results[count] and frees the handle.  Each problem runs the
 * same kernels and decisions as under hot_solve; the slab-pass chunking
 * depends on the launch's total size, so a result is bit-identical to the
 * solo one when the chunking coincides and otherwise differs only in the
 * summation order of column partial sums (within rounding). */
hot_status hot_batch_submit(hot_ctx *ctx, const hot_problem *probs,
                            int32_t count, hot_stream_t stream,
                            hot_batch **out);
hot_status hot_batch_wait(hot_batch *batch, hot_result *results);

/* Continuous-batching service.  A worker thread admits queued problems
 * (FIFO) whenever fewer than max_slots are resident and the sum of their
 * device footprints (hot_ctx_footprint_bytes) stays within hbm_budget_bytes
 * (0: 80% of the free device memory at creation; footprints are computed
 * with the context's launch-shape tuning, and workspaces kept for reuse after
 * a problem finishes count against the budget until they are freed to admit
 * another problem).  Each resident problem is
 * iterated on its own stream by its captured graph, so problems admitted at
 * different times run concurrently; iterates stay on the device until the
 * problem stops.  A problem's result equals its hot_solve result.
 * With HOT_SERVER_SHARED in flags, problems of one precision, one side class
 * (the larger side in 1..32, 33..48, 49..64, 65..96, 97..128, 129..192 or
 * 193..256) and one sigma rule instead share launches: each such class has a
 * group of max_slots slots in one set of device buffers (allocated when the
 * class first appears, counted against the budget, kept until destroy), a
 * problem takes a free slot at the group's next quantum boundary, and every
 * quantum iterates all of the group's problems in the same launches.  A slot
 * keeps the problem's own single-problem geometry, so its result is still
 * bit-identical to hot_solve's.  Problems with HOT_FLAG_ESCALATE, larger
 * sides, or a geometry that does not fit the class's slot run alone as
 * above.  max_slots bounds the resident problems of all kinds together.
 * submit: non-blocking; the histograms (and grid-line positions, if any)
 *   must stay valid until its result has been polled.  HOT_E_INVALID for a malformed problem (histogram values are
 *   validated at admission and reported in the result status), HOT_E_NOMEM
 *   if its footprint alone exceeds the budget.
 * poll: copies up to max finished results (each returned once) with their
 *   tags and latency (submit to completion, seconds); returns how many.
 * drain: waits until every submitted problem has finished (HOT_E_BUSY on
 *   timeout).
 * stats: out[9] = completed, submitted, queued, resident, bytes resident,
 *   most resident at once, p50 latency, p99 latency (seconds), most problems
 *   iterated by one shared launch.
 * cancel: every problem submitted so far ends with HOT_E_CANCELLED (queued
 *   ones at once, resident ones after their current quantum, with their last
 *   iterate's values in the result) unless it has already finished; results
 *   are polled as usual and the server keeps accepting new problems.
 * destroy: drops queued problems, stops resident ones after their current
 *   quantum (their results, not polled, are discarded), frees all. */
#define HOT_SERVER_SHARED 0x1u /* hot_server_config.flags: shared launches */

typedef struct {
  size_t hbm_budget_bytes;
  int32_t max_slots; /* 1..1024 */
  uint32_t flags;    /* HOT_SERVER_* */
} hot_server_config;

hot_status hot_server_create(hot_ctx *ctx, const hot_server_config *cfg,
                             hot_server **out);
hot_status hot_server_submit(hot_server *srv, const hot_problem *prob,
                             uint64_t tag);
int32_t hot_server_poll(hot_server *srv, hot_result *results, uint64_t *tags,
                        double *latency_s, int32_t max);
hot_status hot_server_drain(hot_server *srv, double timeout_s);
hot_status hot_server_stats(hot_server *srv, double *out);
hot_status hot_server_cancel(hot_server *srv);
void hot_server_destroy(hot_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* HOT_H */

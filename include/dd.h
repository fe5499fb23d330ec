/*
 * dd.h -- C-ABI of the MI355X (gfx950) library for entropic domain
 * decomposition of W2 optimal transport between images, after Bonafini &
 * Schmitzer, "Domain decomposition for entropy regularized optimal transport".
 *
 * The problem (eq. "Problem", Sec. 3): for probability images mu, nu on the
 * same H x W pixel grid and c(x,y) = |x-y|^2 (Sec. 7.1; optionally |x-y|^p,
 * dd_options.cost_p), minimise eps*KL(pi | exp(-c/eps) mu (x) nu) over
 * couplings pi of mu and nu.
 *
 * The state of a problem is the one of Algorithm 2: the Y-marginals nu_i of
 * the plan on every basic cell X_i (s x s pixel blocks) and the X-potentials
 * of the last solve on each composite partition, A (2x2 blocks of basic
 * cells) and B (the same blocks shifted by one basic cell, Sec. 7.1).  One
 * call of dd_half_iterate is one sweep of Algorithm 2 over all cells of one
 * partition: for every composite cell J the cell Y-marginal is assembled from
 * its basic cells, a stabilised Sinkhorn solve (Sec. 6.2) is run from the
 * stored potential, the cell plan is split back into basic-cell marginals,
 * BalanceMeasures and truncation are applied, and the potential is stored.
 *
 * Conventions shared by every call:
 *  - arrays are row-major H x W; level 0 is the coarsest grid (H, W divided
 *    by 2^(n_levels-1)), coarser levels are 2x2 block sums (Sec. 6.4);
 *  - pixel (r,c) of a level with spacing h sits at ((c+1/2)h, (r+1/2)h) in the
 *    unit square, h = 1/max(H,W) on the finest level; eps is in those units;
 *  - potentials are exported as f = eps*log u (absolute units), which is what
 *    an eps change keeps fixed (end of Sec. 6.4);
 *  - basic cells are numbered row-major on the level's basic-cell grid; the
 *    Y-marginal rows hold linear pixel indices r*W+c in increasing order.
 *
 * Ownership and streams: the library copies what it needs at dd_init and
 * owns all device state of a context; export calls write only into buffers
 * the caller provides.  All GPU work of a context is enqueued on
 * dd_options.stream (a hipStream_t, NULL = default stream); calls that return
 * host values synchronise that stream.  A context is not thread-safe.
 *
 * Device memory: the contexts' buffers come from a process-wide cache of
 * device blocks.  A freed buffer (a level change, dd_free) is kept after a
 * device synchronisation and handed out again to a later request of at
 * least half its size on the same device; at most 16 GiB per device are
 * kept, and they stay allocated until the process ends.  A failed
 * allocation releases the device's cache and tries once more.
 *
 * Errors: every call returns a dd_status; negative values are errors and
 * leave a message readable with dd_last_error(ctx).  No exception crosses the
 * ABI.  DD_ENOTCONV (positive) is a warning: some cell hit the Sinkhorn
 * iteration cap even after the safeguard; the iteration still completed.
 */
#ifndef DD_H
#define DD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dd_ctx dd_ctx;

typedef enum {
  DD_OK = 0,
  DD_ENOTCONV = 1,
  DD_EINVAL = -1,
  DD_ENOMEM = -2,
  DD_EHIP = -3,
  DD_ECAPACITY = -4,
  DD_ESTATE = -5
} dd_status;

/* One row of the multi-scale eps schedule (Sec. 7.1 "Multi-scale and
 * eps-scaling"): on `level`, set eps, then run n_half_iters half-iterations
 * starting with partition A.  A stage on a finer level than the current one
 * refines first (dd_refine). */
typedef struct {
  int level;
  double eps;
  int n_half_iters;
} dd_stage;

#define DD_PREC_SPLIT 0
#define DD_PREC_FP64 1

typedef struct {
  double err_tol;          /* Sinkhorn stop: L1 X-marginal error <= err_tol*|mu_J| (Sec. 6.2); default 1e-5 */
  double trunc_threshold;  /* truncation threshold of the basic marginals (Sec. 6.1 (ii)); default 1e-15 */
  int max_sinkhorn_iter;   /* Sinkhorn loop cap per cell solve; default 50000 */
  int safeguard;           /* 1: re-solve failed cells at 2*eps, then eps (Sec. 7.4); default 1 */
  int accel;               /* 1: Chebyshev-accelerated X-iteration of the cell Sinkhorn (same
                              stopping test, same fixed point), 0: plain Sinkhorn; default 1 */
  int newton_after;        /* >0: a cell not converged after this many loops continues with
                              damped Newton steps on its X potential (same stopping test, same
                              fixed point); 0: never; default 384 */
  int precision;           /* DD_PREC_SPLIT (default): FP32 exponentials in the Sinkhorn bulk,
                              FP64 potentials, sums and bookkeeping; DD_PREC_FP64: every cell on
                              the log-domain solver with FP64 exponentials (the arithmetic of the
                              FP64 oracle, for parity runs; slower) */
  int inputs_on_device;    /* 1: mu, nu passed to dd_init are device pointers; default 0 */
  int timing;              /* 1: record HIP events around every kernel of a sweep; default 0 */
  void* stream;            /* hipStream_t for all work of the context; default NULL */
  double cost_p;           /* cost c(x,y) = |x-y|^p, 1 < p <= 16: a cost h(x-y) with h strictly
                              convex (Sec. 7.1, Sec. 8; Monge setting of Sec. 5); default 2,
                              the quadratic cost of the paper's experiments.  eps is in units
                              of that cost (h^p per pixel^p on the unit square) */
  int safeguard_after;     /* >0: a cell not converged after this many loops counts as failing
                              and goes to the safeguard (at most max_sinkhorn_iter); 0: only
                              at max_sinkhorn_iter.  Default 1024: past the Newton budget a
                              cell that has not converged is one whose couplings have nearly
                              vanished (its whole support far from the block), which the
                              doubled eps resolves in a few hundred loops */
} dd_options;

/* Kernels of one sweep (indices of the ms_kernel arrays): 0 cell sizes scan,
 * 1 union, 2 output scan + size bins, 3..7 register solvers for unions of
 * <= 64, 128, 256, 512, 1024 points, 8 streamed solver for unions of <= 8192
 * points, 9 log-domain solver for larger unions, 10 Newton solver for the
 * cells the register and streamed solvers handed over, 11 statistics.
 * Solver bins 0..6 are kernels 3..9; kernels 3..9 run concurrently. */
#define DD_N_KERNELS 12
#define DD_N_BINS 7

typedef struct {
  int n_cells;             /* composite cells solved */
  int loops_max;           /* largest Sinkhorn loop count of a cell */
  int64_t loops_total;     /* sum of Sinkhorn loop counts */
  int n_failed;            /* cells still over the iteration cap after the safeguard */
  int n_safeguard;         /* cells that needed the safeguard */
  int n_newton;            /* cells that switched to Newton steps */
  int64_t nnz;             /* entries of the basic Y-marginals after truncation */
  int64_t entry_evals;     /* sum over cells of loops * |X_J| * |Y_J| (kernel entries touched per loop) */
  double cost;             /* sum over cells of <c, pi_J> (plans before balancing) */
  double obj;              /* sum over cells of eps*KL(pi_J|K_J) - eps*|K_J| */
  double err_x;            /* sum over cells of the L1 X-marginal error */
  double ms;               /* device time of the half-iteration (ms) */
  double ms_kernel[DD_N_KERNELS];   /* per-kernel device time (ms) when timing is on, else 0 */
  double ms_start[DD_N_KERNELS];    /* timing on: start and end of each kernel after the start */
  double ms_end[DD_N_KERNELS];      /* of the sweep (ms; the Newton launches: first start, last end) */
  int cells_bin[DD_N_BINS];         /* cells per solver bin */
  int64_t evals_bin[DD_N_BINS];     /* entry_evals per solver bin: work of that bin's solver
                                       (loops * |X_J| * |Y_J|; for cells handed to a Newton
                                       launch only the loops before the hand-over) */
  int64_t newton_evals;    /* work of the Newton launches: passes over the support (loops and
                              line-search trials) * |X_J| * |Y_J| of the cells handed over */
  int64_t newton_mfma_flops; /* and the FP64 matrix-core flops of their W = Q Q^T formations */
} dd_iter_stats;

typedef struct {
  int n_half_iters;
  int n_cell_solves;
  int64_t loops_total;
  int64_t entry_evals;
  int n_failed;
  int n_safeguard;
  int n_newton;
  int64_t nnz_max;
  double ms_total;         /* wall time of the whole schedule (ms) */
  double ms_kernel[DD_N_KERNELS];   /* summed per-kernel device time when timing is on */
  int launches_bin[DD_N_BINS];      /* solver launches per bin (one per sweep, also when
                                       the bin is empty: such a launch exits at once) */
  int64_t evals_bin[DD_N_BINS];
  int64_t newton_evals;             /* summed over the sweeps as in dd_iter_stats */
  int64_t newton_mfma_flops;
  int newton_launches;              /* Newton launches (four per sweep) */
} dd_run_stats;

typedef struct {
  double cost;             /* <c, pi> of the last half-iteration's cell plans (W2^2 estimate) */
  double obj;              /* eps*KL(pi|K) - eps*|K| of those plans */
  double err_x;            /* L1 error of the X-marginal of those plans */
  double err_y;            /* L1 error of sum_i nu_i against nu (current state) */
  double mass_drift;       /* sum_i | |nu_i| - |mu_i| | (current state) */
  int64_t nnz;
  int level;
  int last_partition;      /* -1 if no half-iteration ran on this level yet */
  double eps;
} dd_cost_report;

/* Export view (two-call protocol): the caller sets the pointers; NULL
 * pointers are skipped.  row_ptr has n_basic+1 entries, col/val nnz,
 * alpha_a/alpha_b H*W of the current level.  Scalar fields are filled by
 * dd_export_plan and read by dd_import_state. */
typedef struct {
  int level;
  int H, W;
  double eps;
  int64_t n_basic;
  int64_t nnz;
  int64_t* row_ptr;
  int32_t* col;
  double* val;
  double* alpha_a;
  double* alpha_b;
} dd_plan_view;

/* Fill *opt with the defaults listed above. */
void dd_options_default(dd_options* opt);

/* Create a problem (eq. "Problem", Algorithm 2 inputs).
 * mu, nu: H x W row-major FP64 probability images (host pointers unless
 *   opt->inputs_on_device); copied, the caller keeps ownership.
 * basic_cell: s, 2 or 4 (a composite cell of 2s x 2s pixels is solved in a
 *   virtual 8x8 block, so s = 2 leaves three quarters of it empty); H and W
 *   must be divisible by 2*s*2^(n_levels-1).  The warm-start network and the
 *   cell features of include/dd_mlp.h need s = 4.
 * schedule: n_stages >= 1 rows, copied; schedule[0].eps is the initial eps.
 * The state starts on level 0 with the product coupling nu_i = |mu_i| nu and
 * zero potentials (Sec. 6.4).  Rejects with DD_EINVAL: non-finite or
 * negative masses, total masses off 1 by more than 1e-9, a basic cell of zero
 * mass, indivisible sizes, eps <= 0, a schedule whose levels decrease.  On
 * success *out owns the context (release with dd_free). */
dd_status dd_init(const double* mu, const double* nu, int height, int width, int basic_cell,
                  int n_levels, const dd_stage* schedule, int n_stages, const dd_options* opt,
                  dd_ctx** out);

/* One sweep of Algorithm 2 over all composite cells of partition 0 (A) or
 * 1 (B) on the current level.  stats (nullable) receives the per-sweep
 * counters; the call synchronises the context stream.  DD_ECAPACITY if the
 * level has more than 2^21 cells in the partition (images above ~11500^2);
 * DD_ESTATE while the context belongs to a batch. */
dd_status dd_half_iterate(dd_ctx* ctx, int partition, dd_iter_stats* stats);

/* Change eps; the potentials f = eps*log u stay as they are (end of Sec. 6.4). */
dd_status dd_set_eps(dd_ctx* ctx, double eps);

/* Coarse-to-fine step (Sec. 6.4): the basic marginals of the next level by
 * eq. (FineBasicMarginals); the potentials of partition A are glued with the
 * help of those of B (the least squares of Sec. 6.3 on the A-cell graph with
 * both orientations of every edge, solved on the device as in
 * dd_certificate), bilinearly interpolated to the fine pixels and used for
 * both partitions.  Allocates and frees device scratch.  DD_ESTATE on the
 * finest level. */
dd_status dd_refine(dd_ctx* ctx);

/* Run the whole schedule given at dd_init from the current state. */
dd_status dd_run_schedule(dd_ctx* ctx, dd_run_stats* stats);

/* FP64 diagnostics (Sec. 7.3 "Solution quality": the transport cost, the
 * L1 marginal errors of X and Y, the sparsity of the basic marginals).
 * err_y, mass_drift and nnz describe the current state; cost, obj and err_x
 * the cell plans of the last half-iteration on this level (the primal
 * iterate of Sec. 6.3), and eps is the eps that half-iteration ran with (the
 * current eps if none ran yet).  Synchronises the context's stream. */
dd_status dd_cost(dd_ctx* ctx, dd_cost_report* report);

/* dd_cost without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same report as dd_cost, computed by the same kernels; their
 * scratch (H*W + 768 doubles) is a static device array of
 * 2^22 + 768 doubles (32 MiB) on every GPU the library runs on, held until
 * the process ends, so the current level may have at most 2^22 pixels
 * (2048 x 2048); larger levels are rejected with DD_ECAPACITY (dd_cost has
 * no such limit).  The array is cleared by a kernel on every call.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (contexts
 * on different streams, other threads) race and must be serialised by the
 * caller.  Allocates nothing on the device or in pinned memory (the host
 * read-back buffer belongs to the context); synchronises the context's
 * stream. */
dd_status dd_cost_noalloc(dd_ctx* ctx, dd_cost_report* report);

/* Export the state (Algorithm 2 outputs) into caller buffers; fills the
 * scalar fields of *view first, so a call with NULL pointers returns sizes. */
dd_status dd_export_plan(dd_ctx* ctx, dd_plan_view* view);

/* Replace the state by view (same level geometry as the context's level
 * view->level; rows sorted, no duplicates); for resume and tests. */
dd_status dd_import_state(dd_ctx* ctx, const dd_plan_view* view);

/* Primal-dual certificate of the current iterate (Sec. 6.3, "Estimating the
 * primal-dual gap"; relative gap of eq. RelPDGap in Sec. 7.3).
 *  - primal = KL(pi|K) - |K| of the last half-iteration's cell plans
 *    (the sum of their cell objectives divided by eps), K = exp(-c/eps) mu nu;
 *  - the X-potentials of the two partitions are glued on the A-cell graph:
 *    every pair of A-cells meeting one B-cell gives an edge in each
 *    orientation with weight log q (mu-weighted means of u_A/u_B and u_B/u_A
 *    over the two overlaps), V minimises sum (V(J2) - V(J1) - log q)^2 with
 *    mean zero (conjugate gradients on the device, relative residual 1e-12
 *    or at most 20 000 steps), alpha_hat = alpha_A + eps V on each A-cell;
 *  - beta_hat is the exact Y-iteration of alpha_hat, summed over the stored
 *    support of the plan (entries below the truncation threshold are left
 *    out, as in the sweeps); then int u_hat v_hat dK = |nu| and
 *    dual = J - |K| = (<alpha_hat, mu> + <beta_hat, nu>)/eps - |nu|;
 *  - gap = primal - dual, rel_gap = gap / primal.
 * alpha_hat and beta_hat: optional host buffers of H*W doubles (NULL to
 * skip); beta_hat is NaN where no stored entry reaches a pixel (counted in
 * n_uncovered; the dual is then not a valid bound).  Synchronises the
 * context's stream.  DD_ESTATE if no half-iteration ran on this level or eps
 * changed after the last one (the primal score belongs to that eps).
 * DD_ENOTCONV (a warning; the report is filled) if the CG solve stopped at
 * its step cap above the residual bound: V is then not the least-squares
 * solution and the dual bounds a less good candidate.
 * Allocates and frees device scratch (4 H*W doubles plus the A-cell graph). */
typedef struct {
  double primal;
  double dual;
  double gap;
  double rel_gap;
  double sum_nu;
  int64_t n_uncovered;
  int n_edges;
  int level;
  double eps;
  int cg_iters;            /* conjugate-gradient steps of the gluing solve */
  double cg_rel_resid;     /* its final residual relative to the right-hand side */
} dd_cert_report;

dd_status dd_certificate(dd_ctx* ctx, dd_cert_report* report, double* alpha_hat,
                         double* beta_hat);

/* Per-cell results of the last half-iteration (arrays of that partition's
 * cell count, cells numbered row-major; nullable): transport cost, objective,
 * X-marginal error, Sinkhorn loops, status (1 cap, 2 non-finite, 4 safeguard). */
dd_status dd_cell_results(dd_ctx* ctx, double* cost, double* obj, double* err_x, int* loops,
                          int* status);

/* Geometry of the current level (all outputs nullable). */
dd_status dd_level_info(const dd_ctx* ctx, int* level, int* height, int* width, int* n_basic,
                        int* n_cells_a, int* n_cells_b, double* eps);

void dd_free(dd_ctx* ctx);

/* Message of the last error on ctx (or of the last failed dd_init when ctx is NULL). */
const char* dd_last_error(const dd_ctx* ctx);

/* ---- Batches of independent problems ----------------------------------
 * The composite cells of one partition are independent subproblems
 * (Algorithm 2), and so are the cells of different problems.  A batch runs
 * the sweeps of several problems together: one set of solver launches per
 * sweep takes the cells of every problem, binned by Y-support size, so that
 * many small images fill the GPU as one large one does.  Each problem keeps
 * its own state, eps, level and schedule; the results are the ones its own
 * dd_half_iterate would give (the kernels and their order per cell are the
 * same).
 *
 * The contexts stay owned by the caller and must outlive the batch; they
 * must share one stream (dd_options.stream).  While the batch exists their
 * own dd_half_iterate and dd_run_schedule return DD_ESTATE (every other call
 * stays valid), and a context belongs to at most one batch.  The network
 * warm start (dd_set_warm_start) is not applied to batched sweeps. */
typedef struct dd_batch dd_batch;

/* Flags of dd_batch_create. */
#define DD_BATCH_GRAPH 1 /* capture the launches of a sweep in a HIP graph and replay
                            it while the sweep's shape (problems, level sizes, buffer
                            capacities) stays the same; the per-problem parameters are
                            read from device memory, refreshed before every replay */

/* Create a batch of n (1 <= n <= 1024) distinct contexts.  DD_EINVAL for a
 * NULL or repeated context, one already in a batch, or mixed streams. */
dd_status dd_batch_create(dd_ctx* const* ctxs, int n, int flags, dd_batch** out);

/* One sweep of partition 0 (A) or 1 (B) over every problem of the batch.
 * stats: NULL or n entries (problem order of dd_batch_create); ms and
 * ms_kernel there are those of the whole batched sweep. */
dd_status dd_batch_half_iterate(dd_batch* batch, int partition, dd_iter_stats* stats);

/* Run every problem's own dd_init schedule from its current stage, in
 * lockstep: sweep t of the batch runs sweep t of every problem that has one
 * left, after that problem's refinements and eps changes; problems whose
 * schedule has ended drop out.  stats: NULL or n entries. */
dd_status dd_batch_run_schedule(dd_batch* batch, dd_run_stats* stats);

/* One step of dd_batch_run_schedule: a single lockstep sweep.  *n_active
 * receives the number of problems that took part (0 once every schedule has
 * ended); stats: NULL or n entries, zero for problems not in the sweep.  A
 * caller can interleave its own work (progress, checkpoints) between steps;
 * a context taken out of the batch resumes its schedule at the start of the
 * stage it was in. */
dd_status dd_batch_schedule_step(dd_batch* batch, dd_iter_stats* stats, int* n_active);

/* Sweeps run and graph captures made by the batch so far (nullable outputs). */
dd_status dd_batch_info(const dd_batch* batch, int* n_problems, long long* n_sweeps,
                        int* n_captures);

/* ---- Launch configuration and autotuning ------------------------------
 * Every solver launch of a sweep loops over a work queue, so its number of
 * workgroups changes the speed, never the result.  A configuration is the
 * number of workgroups per compute unit of each solver launch (1..64,
 * default 8) and of each Newton launch (1..16, default 2). */
typedef struct {
  int solver_per_cu; /* workgroups per solver launch and compute unit, 1..64 (default 8) */
  int newton_per_cu; /* workgroups per Newton launch and compute unit, 1..16 (default 2) */
  int stream_wgs;    /* the streamed solver's workgroups at most, 0..4096 (each re-reads
                        its cell's tile of up to 2 MiB every loop, so fewer of them keep
                        more tiles in the last-level cache); 0 = two per compute unit */
  int cells_per_wg;  /* register solvers: cells a workgroup takes before it exits (then
                        the launch has enough workgroups for every cell, and launches on
                        the other streams get compute units as they finish); 0 = loop
                        until the queue is empty (default) */
  double ms;         /* autotuner: GPU time of the sweep (best of the repetitions) */
} dd_tune_point;

dd_status dd_set_launch(dd_ctx* ctx, const dd_tune_point* cfg);
dd_status dd_batch_set_launch(dd_batch* batch, const dd_tune_point* cfg);
dd_status dd_get_launch(const dd_ctx* ctx, dd_tune_point* cfg);

/* Autotuner: runs the next sweep of `partition` under candidate
 * configurations, reps times each, one axis at a time with the others at the
 * best so far: cells_per_wg 0/1/2/4, stream_wgs 32/64/128/256/0, Newton
 * 1/2/4 and (persistent workgroups only) solver 2/4/8/16 per compute unit
 * (at most 16 distinct points), from the same state (a device snapshot of the basic-cell rows
 * and the partition's potentials, restored before every run and at the end,
 * so the state is unchanged on return), and keeps the fastest for later
 * sweeps.  best: the chosen point; tried (nullable): up to max_tried
 * points in the order run, *n_tried (nullable) their number.  The snapshot
 * needs device memory of the size of the entry buffer. */
dd_status dd_autotune(dd_ctx* ctx, int partition, int reps, dd_tune_point* best,
                      dd_tune_point* tried, int max_tried, int* n_tried);
dd_status dd_batch_autotune(dd_batch* batch, int partition, int reps, dd_tune_point* best,
                            dd_tune_point* tried, int max_tried, int* n_tried);

/* Measured arithmetic peaks of the current device, the denominators of the
 * roofline of the cell solves (the Sinkhorn iteration of the sub-problems,
 * Remark "Sinkhorn algorithm" and Sec. 6.2): the issue rates of the
 * operations the cell solvers are built from (the Sinkhorn loops are FP32
 * multiply-adds on a stored kernel tile, the tile and the Newton steps take
 * FP32 and FP64 exponentials; the roofline of the per-cell loop is the
 * vector ALU, not HBM).  Each rate is the best of three launches of a kernel
 * that runs eight independent dependency chains per thread, eight
 * 256-thread workgroups per compute unit: FP32 fused multiply-adds (not
 * packed; 2 flops each), FP64 fused multiply-adds and FP32 exponentials
 * (v_exp_f32, results per second).  Runs on its own stream of the current
 * device and allocates a small device buffer; returns DD_EINVAL for a null
 * output, DD_EHIP on a HIP error (message: dd_probe_last_error). */
typedef struct {
  double fp32_fma_tflops;  /* FP32 FMA, TFLOP/s */
  double fp64_fma_tflops;  /* FP64 FMA, TFLOP/s */
  double exp_f32_per_s;    /* FP32 exponentials per second */
  int compute_units;       /* of the device */
  double clock_mhz;        /* peak engine clock the runtime reports */
  double ms_fp32, ms_fp64, ms_exp; /* best launch times */
} dd_peaks;

dd_status dd_probe_peaks(dd_peaks* out);
const char* dd_probe_last_error(void);

/* Release the batch (not its contexts, which return to their own sweeps). */
void dd_batch_free(dd_batch* batch);

/* Message of the last error on the batch. */
const char* dd_batch_last_error(const dd_batch* batch);

#ifdef __cplusplus
}
#endif
#endif

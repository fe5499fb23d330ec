/*
 * dd_single.h -- single sparse multi-scale Sinkhorn on the whole grid, the
 * comparison method of Sec. 7.4 ("Comparison to single Sinkhorn algorithm")
 * of Bonafini & Schmitzer: one global Sinkhorn iteration with absorbed
 * (stabilised) potentials, adaptive truncation of the stabilised kernel,
 * a coarse-to-fine scheme and eps-scaling, on the GPU.  It solves the same
 * problem as the domain decomposition of include/dd.h (eq. "Problem"), so
 * the two can be compared on time, kernel entries and dual score.
 *
 * The plan is pi(x,y) = u(x) v(y) exp((alpha(x) + beta(y) - c(x,y))/eps)
 * mu(x) nu(y) on the support where exp((alpha + beta - c)/eps) >= theta
 * (Sec. 7.4: entries of the stabilised kernel below theta = 1e-10 are
 * dropped), recomputed whenever the scalings are absorbed into the
 * potentials.  Each stage of the schedule runs Sinkhorn loops (a Y-iteration,
 * then an X-iteration, Remark "Sinkhorn algorithm") until the X-marginal
 * error after a Y-iteration is at most err_tol (Sec. 7.4 uses the L-infinity
 * error with tolerance 1e-7, taken here as the largest absolute difference
 * max_x |P_X pi(x) - mu(x)| of the unit-mass marginals: the L1 errors the
 * paper's summary table lists for this method, 1e-4 to 3e-3, exceed 1e-7
 * and so rule out a relative reading); a refinement carries the total
 * potentials to the next level by bilinear interpolation.
 *
 * Conventions: as in include/dd.h (row-major H x W FP64 probability images
 * on host memory, pixel centres ((c+1/2)h, (r+1/2)h), h = 1/max(H,W) on the
 * finest level, levels by 2x2 block sums, eps in unit coordinates; the cost
 * c = |x-y|^cost_p).  Only the dd_stage fields level and eps are used.
 *
 * Errors: DD_EINVAL for bad arguments (sizes not divisible by
 * 2^(n_levels-1), masses not summing to 1, bad schedule or options),
 * DD_ENOMEM, DD_EHIP; DD_ENOTCONV (report filled) when a stage hit max_iter
 * or a row or column of positive mass lost its whole kernel support (the
 * failure the paper reports for this method at large sizes).
 * Synchronises opt->stream; allocates and frees its own device memory.
 */
#ifndef DD_SINGLE_H
#define DD_SINGLE_H
#include <stdint.h>

#include "dd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DD_SINGLE_LINF 0 /* stop on max |P_X pi - mu| <= err_tol */
#define DD_SINGLE_L1 1   /* stop on sum |P_X pi - mu| <= err_tol */

typedef struct {
  double err_tol;   /* default 1e-7 */
  int err_norm;     /* DD_SINGLE_LINF (default) or DD_SINGLE_L1 */
  double theta;     /* kernel truncation threshold, default 1e-10 */
  double absorb;    /* absorb when max |log u| or |log v| exceeds this, default 30 */
  int max_iter;     /* Sinkhorn loops per stage at most, default 200000 */
  int check_every;  /* loops between error checks (and absorption tests), default 16 */
  double cost_p;    /* c = |x-y|^p, 1 < p <= 16, default 2 */
  void* stream;     /* hipStream_t, default NULL */
} dd_single_options;

typedef struct {
  int n_stages;
  int level;               /* level of the result (the last stage's) */
  double eps;
  int64_t loops_total;     /* Sinkhorn loops over the schedule */
  int loops_max_stage;
  int n_absorb;            /* absorptions within stages (each recomputes the support) */
  int64_t entries_max;     /* kernel support size (entries >= theta), largest over the schedule */
  int64_t entries_final;   /* and at the last support computation */
  int64_t entry_evals;     /* kernel entries evaluated by all passes (box areas) */
  double err_x_l1;         /* X-marginal errors of the final plan */
  double err_x_linf;
  double err_y_l1;         /* Y-marginal error (zero up to rounding: the last step is a Y-iteration) */
  double cost;             /* <c, pi> */
  double primal;           /* KL(pi|K) - |K| of the final plan, K = exp(-c/eps) mu nu */
  double dual;             /* J(u, v) - |K| of the final potentials (eq. EntropicOTDualObjective,
                              the kernel integral taken over the support) */
  double plan_mass;
  double ms;               /* wall time of the call */
  int failed;
} dd_single_report;

void dd_single_options_default(dd_single_options* opt);

/* Solve; alpha_out / beta_out (nullable, H*W doubles) receive the total
 * potentials eps log(u) + alpha and eps log(v) + beta of the last level. */
dd_status dd_single_solve(const double* mu, const double* nu, int height, int width,
                          int n_levels, const dd_stage* schedule, int n_stages,
                          const dd_single_options* opt, dd_single_report* report,
                          double* alpha_out, double* beta_out);

/* Message of the last failed dd_single_solve of the calling thread. */
const char* dd_single_last_error(void);

#ifdef __cplusplus
}
#endif
#endif

/*
 * ddo.h -- FP64 CPU oracle of entropic domain decomposition for W2 optimal
 * transport between images (Bonafini & Schmitzer, "Domain decomposition for
 * entropy regularized optimal transport").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this library; it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can check the GPU path against a plain,
 * slow, obviously correct implementation of the same iteration.
 *
 * All pointers are host pointers.  Every function returns 0 on success and a
 * negative code on error (-1 invalid argument, -2 out of memory, -5 state);
 * ddo_half_iterate returns 1 when some cell hit the iteration cap.
 * Per-cell status bits: 1 cap, 2 non-finite, 4 safeguard used, 8 skipped (mask),
 * 16 Newton steps used.
 *
 * Conventions (the readings of the paper this oracle implements):
 *  - level 0 is the coarsest grid, level nlev-1 the finest; each coarser
 *    level is the 2x2 block-sum push-forward of the next finer one (Sec. 6.4).
 *  - pixel (r,c) of a level with spacing h sits at ((c+1/2)h, (r+1/2)h);
 *    c(x,y) = |x-y|^2 (Sec. 7.1).  h = 1/max(H,W) at the finest level and
 *    doubles per coarser level.  Optionally c(x,y) = |x-y|^p, p > 1.
 *  - basic cells are s x s pixel blocks; partition A groups 2x2 basic cells,
 *    partition B the same offset by one basic cell (Sec. 7.1).  Basic cells
 *    in a composite cell are ordered row-major, pixels in a basic cell too.
 *  - potentials alpha_A, alpha_B are stored per pixel as f = eps*log u (the
 *    dual variable in absolute units), so an eps change leaves them as they
 *    are (end of Sec. 6.4).
 */
#ifndef DDO_H
#define DDO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddo_ctx ddo_ctx;

typedef struct {
  double err_tol;    /* Sinkhorn stop: L1 X-marginal error <= err_tol*|mu_J| (Sec. 6.2) */
  double trunc;      /* truncation threshold theta (Sec. 6.1 item ii) */
  int max_iter;      /* Sinkhorn loop cap per cell solve */
  int n_threads;     /* OpenMP threads over cells (0 = runtime default) */
  int safeguard;     /* 1: re-solve failed cells at 2*eps, then eps (Sec. 7.4) */
  int accel;         /* 1: Chebyshev-accelerated X-iteration, 0: plain Sinkhorn */
  int newton_after;  /* >0: switch a cell to Newton steps after this many loops; 0: never */
  double cost_p;     /* c(x,y) = |x-y|^p, p > 1 (Sec. 7.1: h(x-y), h strictly convex); 0 = 2 */
  int safeguard_after; /* >0: a cell not converged after this many loops counts as failing
                          and goes to the safeguard (capped by max_iter); 0: at max_iter */
} ddo_opts;

typedef struct {
  int level;
  double eps;
  int n_half;        /* half-iterations in this stage, starting with partition A */
} ddo_stage;

typedef struct {
  int n_cells;
  int64_t loops_total;
  int loops_max;
  int n_failed;      /* cells that hit max_iter or went non-finite (after safeguard) */
  int n_safeguard;   /* cells that needed the safeguard */
  int n_newton;      /* cells that switched to Newton steps */
  int64_t nnz;       /* entries of the basic Y-marginals after truncation */
  double cost;       /* sum over cells of <c, pi_J> (plans before balance/truncation) */
  double obj;        /* sum over cells of eps*KL(pi_J|K_J) - eps*|K_J| */
  double err_x;      /* sum over cells of the L1 X-marginal error */
} ddo_iter_stats;

typedef struct {
  double cost, obj, err_x, err_y, mass_drift;
  int64_t nnz;
  int level, last_partition;
  double eps;
} ddo_cost_report;

int ddo_init(const double* mu, const double* nu, int H, int W, int s, int nlev,
             double eps, const ddo_opts* opt, ddo_ctx** out);
void ddo_free(ddo_ctx* c);
int ddo_set_eps(ddo_ctx* c, double eps);
int ddo_half_iterate(ddo_ctx* c, int partition, const uint8_t* cell_mask, ddo_iter_stats* st);
int ddo_refine(ddo_ctx* c);
int ddo_run_schedule(ddo_ctx* c, const ddo_stage* st, int n, ddo_iter_stats* total);
int ddo_cost(ddo_ctx* c, ddo_cost_report* r);

/* geometry of the current level */
int ddo_level_info(const ddo_ctx* c, int* level, int* H, int* W, int* n_basic,
                   int* n_cells_a, int* n_cells_b, double* eps, double* h);
/* basic-cell ids of the cells of a partition: cells[k*4+q] (-1 padded) */
int ddo_cells(const ddo_ctx* c, int partition, int* cells);

/* two-call export: pass NULL arrays to get nnz; then fill.
 * row_ptr: n_basic+1, col/val: nnz, alpha_a/alpha_b: H*W of the current level */
int ddo_export(const ddo_ctx* c, int64_t* nnz, int64_t* row_ptr, int32_t* col,
               double* val, double* alpha_a, double* alpha_b);
/* replace the state of the current level (rows sorted, no duplicates) */
int ddo_import(ddo_ctx* c, int level, double eps, const int64_t* row_ptr,
               const int32_t* col, const double* val, const double* alpha_a,
               const double* alpha_b);
/* per-cell results of the last half-iteration (arrays of n_cells of that partition) */
int ddo_cell_results(const ddo_ctx* c, double* cost, double* obj, double* err_x,
                     int* loops, int* status);

/* One composite-cell problem, for unit tests: log-domain Sinkhorn between
 * mu (nx points at integer coords xr,xc) and nu (ny points at yr,yc) with
 * cost lam*|dx|^2 in units of eps (lam = h^2/eps), optionally accelerated
 * and with the Newton fallback after newton_after loops.  F (in/out, units of
 * eps) is the warm start; on return G holds the Y potential of the last
 * Y-update and plan (nx*ny, row-major by x) the plan of that Y-update.
 * Returns 0 converged, 1 at the cap, 2 non-finite, +16 when Newton ran. */
/* the same with c = lam*|x-y|^cost_p, cost_p > 1 */
int ddo_cell_solve_p(int nx, const int* xr, const int* xc, const double* mu,
                     int ny, const int* yr, const int* yc, const double* nu,
                     double lam, double cost_p, double tol, int max_iter, int accel,
                     int newton_after, double* F, double* G, double* plan, int* loops,
                     double* err);
int ddo_cell_solve(int nx, const int* xr, const int* xc, const double* mu,
                   int ny, const int* yr, const int* yc, const double* nu,
                   double lam, double tol, int max_iter, int accel, int newton_after,
                   double* F, double* G, double* plan, int* loops, double* err);

#ifdef __cplusplus
}
#endif
#endif

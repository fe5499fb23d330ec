/*
 * ddo.c -- FP64 CPU oracle of entropic domain decomposition (test
 * infrastructure only; see ddo.h).  Plain loops, FP64 everywhere, OpenMP over
 * the independent composite cells of a partition.  Written from the paper:
 *
 *   Algorithm 2 (practical entropic domain decomposition) for one partition
 *   sweep; Remark "Sinkhorn algorithm" and Sec. 6.2 for the cell solver and
 *   its stopping rule; Sec. 6.2 for BalanceMeasures; Sec. 6.1 (ii) for
 *   truncation; Sec. 6.3 for gluing cell duals; Sec. 6.4, eq.
 *   (FineBasicMarginals) for coarse-to-fine refinement; Sec. 7.1 for the
 *   partitions and the W2 cost.
 *
 * Readings where the paper leaves a choice open are marked READING and are
 * listed with their reasons in the design notes of the repository.
 */
#include "ddo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
  int H, W, bh, bw;
  double h;
  double *mu, *nu;
} lvl_t;

typedef struct {
  int nq;
  int q[4];
} cell_t;

struct ddo_ctx {
  int nlev, s, lev;
  lvl_t* L;
  double eps;
  ddo_opts opt;
  int nb;
  int64_t* rp;
  int32_t* col;
  double* val;
  double *aA, *aB;
  int nc[2];
  cell_t* cells[2];
  int last_part, rc_n;
  double *rc_cost, *rc_obj, *rc_err;
  int *rc_loops, *rc_status;
};

/* ------------------------------------------------------------------ cells */

/* Partition A: 2x2 blocks of basic cells.  Partition B: the same blocks
 * shifted by one basic cell, so row groups are {0},{1,2},...,{bh-1}
 * (Sec. 7.1, "Basic and composite partitions"). */
static int group_count(int nbasic, int part) { return part == 0 ? nbasic / 2 : nbasic / 2 + 1; }
static void group_members(int nbasic, int part, int g, int* lo, int* n) {
  if (part == 0) {
    *lo = 2 * g;
    *n = 2;
  } else {
    int a = 2 * g - 1, b = 2 * g;
    if (a < 0) a = 0;
    if (b > nbasic - 1) b = nbasic - 1;
    *lo = a;
    *n = b - a + 1;
  }
}

static cell_t* build_cells(int bh, int bw, int part, int* ncell) {
  int gr = group_count(bh, part), gc = group_count(bw, part);
  cell_t* cs = (cell_t*)malloc(sizeof(cell_t) * (size_t)gr * gc);
  if (!cs) return NULL;
  int k = 0;
  for (int i = 0; i < gr; i++) {
    int r0, nr;
    group_members(bh, part, i, &r0, &nr);
    for (int j = 0; j < gc; j++) {
      int c0, ncc;
      group_members(bw, part, j, &c0, &ncc);
      cell_t* C = &cs[k++];
      C->nq = 0;
      for (int a = 0; a < 4; a++) C->q[a] = -1;
      for (int a = 0; a < nr; a++)
        for (int b = 0; b < ncc; b++) C->q[C->nq++] = (r0 + a) * bw + (c0 + b);
    }
  }
  *ncell = k;
  return cs;
}

static int rebuild_cells(ddo_ctx* c) {
  lvl_t* l = &c->L[c->lev];
  for (int p = 0; p < 2; p++) {
    free(c->cells[p]);
    c->cells[p] = build_cells(l->bh, l->bw, p, &c->nc[p]);
    if (!c->cells[p]) return -2;
  }
  c->nb = l->bh * l->bw;
  return 0;
}

/* pixel k (0..s*s*nq-1) of a composite cell -> (row, col) */
static void cell_pixel(const lvl_t* l, int s, const cell_t* C, int k, int* r, int* cc) {
  int q = k / (s * s), p = k % (s * s);
  int b = C->q[q];
  int br = b / l->bw, bc = b % l->bw;
  *r = br * s + p / s;
  *cc = bc * s + p % s;
}

/* --------------------------------------------------------------- Sinkhorn */

/* Chebyshev acceleration of the X-iteration (optional).  One Sinkhorn loop
 * F -> X(Y(F)) is a fixed-point map whose Jacobian at the solution has real
 * eigenvalues in [0, rho) (it is similar to a symmetric positive
 * semi-definite matrix), so the Chebyshev semi-iterative method for the
 * interval [0, rho] (Golub & Varga 1961) converges at the rate
 * (1 - sqrt(1 - rho)) / (1 + sqrt(1 - rho)) instead of rho.  The Y-iteration
 * stays exact, so the stopping test (X-marginal error after a Y-iteration)
 * and the exact Y-marginal at termination are those of Sec. 6.2.  The same
 * rule (constants and decisions) runs in the GPU solvers. */
typedef struct {
  double rho, omega, hist[17];
  int k, kstart, pstart, att;
} cheb_t;

static void cheb_reset(cheb_t* c) {
  memset(c, 0, sizeof(*c));
  c->rho = -1;
}

/* decide the update after loop `it` (1-based) with error err; returns 0 for
 * a plain step F <- Fh, 1 for a Chebyshev step with weights (*a, *b, *d):
 * F <- a F + b Fh + d Fprev.  Plain loops estimate rho from the error decay
 * over the last 8 loops (at least 16 plain loops after a (re)start); a
 * Chebyshev run that decays slower than the square root of its promised
 * rate over a 16-loop window is abandoned for plain loops; at most four
 * runs per solve, rho <= 0.9999, so the solver always ends as plain
 * Sinkhorn if acceleration does not pay. */
static int cheb_next(cheb_t* c, int it, double err, double* a, double* b, double* d) {
  c->hist[it % 17] = err;
  if (c->rho < 0) {
    if (it - c->pstart >= 16 && c->att < 4) {
      double r = pow(err / c->hist[(it - 8) % 17], 1.0 / 8);
      if (r > 0.8) {
        c->rho = r < 0.9999 ? r : 0.9999;
        c->k = 0;
        c->kstart = it;
        c->att++;
      }
    }
    return 0;
  }
  if (it - c->kstart >= 16 && (it - c->kstart) % 16 == 0) {
    double robs = pow(err / c->hist[(it - 16) % 17], 1.0 / 16);
    double sq = sqrt(1 - c->rho), cexp = (1 - sq) / (1 + sq);
    if (robs > sqrt(cexp)) {
      c->rho = -1;
      c->pstart = it;
      return 0;
    }
  }
  double sigma = c->rho / (2 - c->rho), gamma = 2 / (2 - c->rho);
  if (c->k == 0)
    c->omega = 1;
  else if (c->k == 1)
    c->omega = 1 / (1 - sigma * sigma / 2);
  else
    c->omega = 1 / (1 - sigma * sigma * c->omega / 4);
  c->k++;
  *a = c->omega * (1 - gamma);
  *b = c->omega * gamma;
  *d = 1 - c->omega;
  return 1;
}

/* Newton fallback for slowly converging cells (optional, after a fixed
 * number of Sinkhorn loops).  The cell problem of Remark "Sinkhorn algorithm"
 * is maximised over the X potential alone, the Y potential being eliminated
 * by the exact Y-iteration (the semi-dual):
 *
 *   Phi(F) = sum_x mu(x) F(x) - sum_y nu(y) L_y(F),
 *   L_y(F) = log sum_x exp(F(x) - C(x,y)) mu(x),
 *
 * with p_x(y) = exp(F(x) - C(x,y)) mu(x) / exp(L_y) the conditional plan, so
 * that pi(x,y) = nu(y) p_x(y) is the plan after a Y-iteration.  Its gradient
 * is mu - r (r the X-marginal of pi) and minus its Hessian is the graph
 * Laplacian of the weights W(x,x') = sum_y nu(y) p_x(y) p_x'(y).  A slowly
 * converging Sinkhorn iteration means that this graph is nearly disconnected
 * (a tiny Laplacian eigenvalue); the Newton step resolves exactly that mode.
 * The stopping test is the one of Sec. 6.2 (X-marginal error after a
 * Y-iteration), so the fixed point and the exact Y-marginal at termination are
 * those of the Sinkhorn solver.  The same rule (constants and decisions) runs
 * in the GPU solvers. */
#define NEWTON_MAX_STEPS 100
#define NEWTON_STEP_CAP 8.0
#define NEWTON_TRIALS 10
#define NEWTON_ARMIJO 1e-4

/* Solve Lap(W) d = b with d[n-1] = 0 (b must sum to zero) by Gaussian
 * elimination in the subtraction-free form of Grassmann, Taksar and Heyman:
 * the Schur complement of a graph Laplacian is the Laplacian of the weights
 * W(i,j) + W(i,k) W(k,j) / d_k, and every pivot d_k is taken as the sum of the
 * remaining off-diagonal weights of its row, so tiny eigenvalues keep their
 * relative accuracy.  W (n*n, row-major, diagonal ignored) is overwritten. */
static void gth_solve(int n, double* W, double* b, double* d, double* piv) {
  for (int k = 0; k < n - 1; k++) {
    double dk = 0;
    for (int j = k + 1; j < n; j++) dk += W[(size_t)k * n + j];
    piv[k] = dk;
    if (!(dk > 0)) continue;
    for (int i = k + 1; i < n; i++) {
      double c = W[(size_t)i * n + k] / dk;
      if (c == 0) continue;
      b[i] += c * b[k];
      for (int j = k + 1; j < n; j++)
        if (j != i) W[(size_t)i * n + j] += c * W[(size_t)k * n + j];
    }
  }
  d[n - 1] = 0;
  for (int k = n - 2; k >= 0; k--) {
    double s = b[k];
    for (int j = k + 1; j < n; j++) s += W[(size_t)k * n + j] * d[j];
    d[k] = piv[k] > 0 ? s / piv[k] : 0.0;
  }
}

/* e^b - 1 - b >= 0 without cancellation for small |b| */
static double phi1(double b) {
  if (fabs(b) < 1e-3) return b * b * (0.5 + b * (1.0 / 6 + b * (1.0 / 24 + b / 120)));
  return expm1(b) - b;
}

/* Cost of moving mass between pixels (dr, dc) apart, in units of h^p:
 * c(x,y) = h(x - y) with h(z) = |z|^p, p > 1 strictly convex (Sec. 7.1; the
 * quadratic cost p = 2 is the paper's experiments, exact in integers). */
static double cost_units(double dr, double dc, double p) {
  double d2 = dr * dr + dc * dc;
  if (p == 2.0) return d2;
  return d2 > 0 ? pow(d2, 0.5 * p) : 0.0;
}

/* Newton iterations from F (loops it0+1 ...); same outputs as sinkhorn_log.
 * Each iteration is one Y-iteration (a loop), the stopping test, then either
 * a damped Newton step or, when the line search fails or after
 * NEWTON_MAX_STEPS steps, a plain X-iteration.
 *   direction: Lap(W) d = g - r sum(g)/sum(r), g = mu - r (the projection
 *     makes the right side sum to zero; d is grounded at the last active x),
 *     scaled down to max|d| <= NEWTON_STEP_CAP;
 *   line search: t = 1, 1/2, ... (NEWTON_TRIALS values), accept when
 *     Phi(F + t d) - Phi(F) >= NEWTON_ARMIJO t <g, d>, where the increase is
 *     evaluated from the conditional plans at F as
 *     <g, a> - sum_y nu(y) log(sum_x p_x(y) exp(a(x) - c_y)), a = t d,
 *     c_y = sum_x p_x(y) a(x) -- both terms are non-negative sums, so the
 *     test stays meaningful when the increase is far below the size of Phi. */
static int newton_log(int nx, const int* xr, const int* xc, const double* mu, int ny,
                      const int* yr, const int* yc, const double* nu, double lam, double cp,
                      double tol,
                      int it0, int maxit, double* F, double* G, int* loops, double* err_out) {
  int n = 0;
  for (int i = 0; i < nx; i++) n += mu[i] > 0;
  int* act = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
  double* P = malloc(sizeof(double) * (size_t)n * ny);
  double* W = malloc(sizeof(double) * (size_t)n * n);
  double* buf = malloc(sizeof(double) * (size_t)n * 6);
  if (!act || !P || !W || !buf || n == 0) {
    free(act);
    free(P);
    free(W);
    free(buf);
    *loops = it0;
    return 2;
  }
  double *r = buf, *g = buf + n, *b = buf + 2 * n, *dd = buf + 3 * n, *piv = buf + 4 * n,
         *lm = buf + 5 * n;
  n = 0;
  for (int i = 0; i < nx; i++)
    if (mu[i] > 0) {
      act[n] = i;
      lm[n] = log(mu[i]);
      n++;
    }
  int it = it0, rc = 1, nst = 0;
  double err = INFINITY;
  while (it < maxit) {
    it++;
    /* Y-iteration and conditional plans */
    for (int j = 0; j < ny; j++) {
      double m = -INFINITY;
      for (int a = 0; a < n; a++) {
        int i = act[a];
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        double e = F[i] + lm[a] - lam * cost_units(dr, dc, cp);
        if (e > m) m = e;
      }
      double s = 0;
      for (int a = 0; a < n; a++) {
        int i = act[a];
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        double v = exp(F[i] + lm[a] - lam * cost_units(dr, dc, cp) - m);
        P[(size_t)a * ny + j] = v;
        s += v;
      }
      for (int a = 0; a < n; a++) P[(size_t)a * ny + j] /= s;
      G[j] = -(m + log(s));
    }
    err = 0;
    for (int a = 0; a < n; a++) {
      double s = 0;
      for (int j = 0; j < ny; j++) s += nu[j] * P[(size_t)a * ny + j];
      r[a] = s;
      err += fabs(s - mu[act[a]]);
    }
    if (!isfinite(err)) {
      rc = 2;
      break;
    }
    if (err <= tol) {
      rc = 0;
      break;
    }
    if (it >= maxit) break;
    int step = 0;
    double t = 1, slope = 0;
    if (nst < NEWTON_MAX_STEPS && n > 1) {
      nst++;
      for (int a = 0; a < n; a++)
        for (int c = 0; c < n; c++) {
          double s = 0;
          if (a != c)
            for (int j = 0; j < ny; j++) s += nu[j] * P[(size_t)a * ny + j] * P[(size_t)c * ny + j];
          W[(size_t)a * n + c] = s;
        }
      double sg = 0, sr = 0;
      for (int a = 0; a < n; a++) {
        g[a] = mu[act[a]] - r[a];
        sg += g[a];
        sr += r[a];
      }
      for (int a = 0; a < n; a++) b[a] = g[a] - r[a] * (sg / sr);
      gth_solve(n, W, b, dd, piv);
      double dm = 0;
      for (int a = 0; a < n; a++) dm = fmax(dm, fabs(dd[a]));
      if (dm > NEWTON_STEP_CAP)
        for (int a = 0; a < n; a++) dd[a] *= NEWTON_STEP_CAP / dm;
      for (int a = 0; a < n; a++) slope += g[a] * dd[a];
      if (slope > 0) {
        for (int trial = 0; trial < NEWTON_TRIALS; trial++) {
          double inc = 0;
          for (int a = 0; a < n; a++) inc += g[a] * t * dd[a];
          for (int j = 0; j < ny; j++) {
            double cy = 0, s = 0;
            for (int a = 0; a < n; a++) cy += P[(size_t)a * ny + j] * t * dd[a];
            for (int a = 0; a < n; a++) s += P[(size_t)a * ny + j] * phi1(t * dd[a] - cy);
            inc -= nu[j] * log1p(s);
          }
          if (inc >= NEWTON_ARMIJO * t * slope) {
            step = 1;
            break;
          }
          t *= 0.5;
        }
      }
    }
    if (step) {
      for (int a = 0; a < n; a++) F[act[a]] += t * dd[a];
    } else {
      /* plain X-iteration: F <- F + log mu - log r */
      for (int a = 0; a < n; a++) F[act[a]] += lm[a] - log(r[a]);
    }
  }
  *loops = it;
  *err_out = err;
  free(act);
  free(P);
  free(W);
  free(buf);
  return rc;
}

/* Log-domain Sinkhorn of Remark "Sinkhorn algorithm", in the dual variables
 * F = f/eps, G = g/eps, with plan pi(x,y) = exp(F(x)+G(y)-C(x,y)) mu(x) nu(y)
 * and C = lam*|x-y|^p (integer pixel offsets, cost_units).  Warm start F, first a
 * Y-iteration; after each Y-iteration the L1 error of the X-marginal is
 * checked and the solver stops there, so the Y-marginal holds exactly
 * (Sec. 6.2).  Returns 0 when converged, 1 at the iteration cap, 2 when a
 * value went non-finite. */
static int sinkhorn_log(int nx, const int* xr, const int* xc, const double* mu,
                        int ny, const int* yr, const int* yc, const double* nu,
                        double lam, double cp, double tol, int maxit, int accel,
                        int newton_after,
                        double* F, double* G, double* Fh, int* loops, double* err_out,
                        int* used_newton) {
  double* lmu = (double*)malloc(sizeof(double) * (size_t)nx);
  double* lnu = (double*)malloc(sizeof(double) * (size_t)ny);
  double* Fp = (double*)malloc(sizeof(double) * (size_t)nx);
  if (!lmu || !lnu || !Fp) {
    free(lmu);
    free(lnu);
    free(Fp);
    return 2;
  }
  for (int i = 0; i < nx; i++) lmu[i] = mu[i] > 0 ? log(mu[i]) : -INFINITY;
  for (int j = 0; j < ny; j++) lnu[j] = nu[j] > 0 ? log(nu[j]) : -INFINITY;
  for (int i = 0; i < nx; i++) Fp[i] = F[i];
  cheb_t ch;
  cheb_reset(&ch);
  int rc = 1;
  double err = INFINITY;
  int it;
  for (it = 1; it <= maxit; it++) {
    /* Y-iteration: G(y) = -log sum_x exp(F(x) - C(x,y)) mu(x) */
    for (int j = 0; j < ny; j++) {
      double m = -INFINITY;
      for (int i = 0; i < nx; i++) {
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        double e = F[i] + lmu[i] - lam * cost_units(dr, dc, cp);
        if (e > m) m = e;
      }
      double s = 0;
      for (int i = 0; i < nx; i++) {
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        s += exp(F[i] + lmu[i] - lam * cost_units(dr, dc, cp) - m);
      }
      G[j] = -(m + log(s));
    }
    /* X-marginal of the current plan: mu(x) exp(F(x) - Fh(x)) with
     * Fh(x) = -log sum_y exp(G(y) - C(x,y)) nu(y) */
    err = 0;
    for (int i = 0; i < nx; i++) {
      double m = -INFINITY;
      for (int j = 0; j < ny; j++) {
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        double e = G[j] + lnu[j] - lam * cost_units(dr, dc, cp);
        if (e > m) m = e;
      }
      double s = 0;
      for (int j = 0; j < ny; j++) {
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        s += exp(G[j] + lnu[j] - lam * cost_units(dr, dc, cp) - m);
      }
      Fh[i] = -(m + log(s));
      if (mu[i] > 0) err += mu[i] * fabs(exp(F[i] - Fh[i]) - 1.0);
    }
    if (!isfinite(err)) {
      rc = 2;
      break;
    }
    if (err <= tol) {
      rc = 0;
      break;
    }
    if (it == maxit) break;
    /* X-iteration (plain, or the Chebyshev-accelerated one) */
    double a = 0, b = 1, d = 0;
    int acc = accel ? cheb_next(&ch, it, err, &a, &b, &d) : 0;
    for (int i = 0; i < nx; i++)
      if (mu[i] > 0) {
        double fn = acc ? a * F[i] + b * Fh[i] + d * Fp[i] : Fh[i];
        Fp[i] = F[i];
        F[i] = fn;
      }
    if (it == newton_after) {
      free(lmu);
      free(lnu);
      free(Fp);
      *used_newton = 1;
      return newton_log(nx, xr, xc, mu, ny, yr, yc, nu, lam, cp, tol, it, maxit, F, G, loops,
                        err_out);
    }
  }
  if (it > maxit) it = maxit;
  *loops = it;
  *err_out = err;
  free(lmu);
  free(lnu);
  free(Fp);
  return rc;
}

int ddo_cell_solve_p(int nx, const int* xr, const int* xc, const double* mu, int ny,
                     const int* yr, const int* yc, const double* nu, double lam, double cost_p,
                     double tol, int max_iter, int accel, int newton_after, double* F,
                     double* G, double* plan, int* loops, double* err) {
  if (nx <= 0 || ny <= 0 || !(lam > 0) || max_iter < 1 || !(cost_p > 1)) return -1;
  double* Fh = (double*)malloc(sizeof(double) * (size_t)nx);
  if (!Fh) return -2;
  int used = 0;
  const double cp = cost_p;
  int rc = sinkhorn_log(nx, xr, xc, mu, ny, yr, yc, nu, lam, cp, tol, max_iter, accel,
                        newton_after, F, G, Fh, loops, err, &used);
  free(Fh);
  if (used && rc >= 0) rc += 16;
  if (plan) {
    for (int i = 0; i < nx; i++)
      for (int j = 0; j < ny; j++) {
        double dr = xr[i] - yr[j], dc = xc[i] - yc[j];
        plan[(size_t)i * ny + j] =
            (mu[i] > 0 && nu[j] > 0)
                ? exp(F[i] + G[j] - lam * cost_units(dr, dc, cp)) * mu[i] * nu[j]
                : 0.0;
      }
  }
  return rc;
}

int ddo_cell_solve(int nx, const int* xr, const int* xc, const double* mu, int ny,
                   const int* yr, const int* yc, const double* nu, double lam,
                   double tol, int max_iter, int accel, int newton_after, double* F,
                   double* G, double* plan, int* loops, double* err) {
  return ddo_cell_solve_p(nx, xr, xc, mu, ny, yr, yc, nu, lam, 2.0, tol, max_iter, accel,
                          newton_after, F, G, plan, loops, err);
}

/* ------------------------------------------------------------ one cell */

typedef struct {
  int nq;
  int n[4];
  int32_t* col[4];
  double* val[4];
  double cost, obj, err;
  int loops, status;
} cell_out_t;

/* Sorted union of the Y-supports of the basic cells of J, with
 * nu_J = sum_i nu_i (Algorithm 2, "compute Y-marginal on cell").
 * Duplicates are summed in basic-cell order. */
static int cell_union(const ddo_ctx* c, const cell_t* C, int32_t** ys, double** nuJ) {
  int64_t tot = 0;
  for (int q = 0; q < C->nq; q++) tot += c->rp[C->q[q] + 1] - c->rp[C->q[q]];
  int32_t* Y = (int32_t*)malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
  double* V = (double*)malloc(sizeof(double) * (size_t)(tot > 0 ? tot : 1));
  if (!Y || !V) {
    free(Y);
    free(V);
    return -1;
  }
  int64_t pos[4], end[4];
  for (int q = 0; q < C->nq; q++) {
    pos[q] = c->rp[C->q[q]];
    end[q] = c->rp[C->q[q] + 1];
  }
  int n = 0;
  for (;;) {
    int32_t key = INT32_MAX;
    int any = 0;
    for (int q = 0; q < C->nq; q++)
      if (pos[q] < end[q] && c->col[pos[q]] <= key) {
        key = c->col[pos[q]];
        any = 1;
      }
    if (!any) break;
    double v = 0;
    for (int q = 0; q < C->nq; q++)
      if (pos[q] < end[q] && c->col[pos[q]] == key) {
        v += c->val[pos[q]];
        pos[q]++;
      }
    Y[n] = key;
    V[n] = v;
    n++;
  }
  *ys = Y;
  *nuJ = V;
  return n;
}

/* BalanceMeasures (Sec. 6.2).  The paper fixes only its properties: after
 * it |nu_i| = |mu_i|, nu_i >= 0, sum_i nu_i unchanged pointwise, no new
 * support points.  READING: with d_i = |mu_i| - |nu_i|, E = sum of -d_i over
 * d_i<0 (excess), D = sum of d_i over d_i>0 (deficit), T = min(E,D): every
 * excess cell a gives up the fraction t_a = T(-d_a)/(E |nu_a|) of its mass at
 * every y, and the freed mass R(y) is handed to the deficit cells b in the
 * proportions d_b/D. */
static void balance(int nq, int ny, double* const* nuq, const double* mass_mu) {
  double d[4], E = 0, D = 0, nrm[4];
  for (int q = 0; q < nq; q++) {
    double s = 0;
    for (int j = 0; j < ny; j++) s += nuq[q][j];
    nrm[q] = s;
    d[q] = mass_mu[q] - s;
    if (d[q] < 0) E += -d[q];
    if (d[q] > 0) D += d[q];
  }
  double T = E < D ? E : D;
  if (!(T > 0)) return;
  double t[4];
  for (int q = 0; q < nq; q++) t[q] = d[q] < 0 ? T * (-d[q]) / (E * nrm[q]) : 0.0;
  for (int j = 0; j < ny; j++) {
    double R = 0;
    for (int q = 0; q < nq; q++)
      if (d[q] < 0) {
        double r = nuq[q][j] * t[q];
        nuq[q][j] -= r;
        R += r;
      }
    for (int q = 0; q < nq; q++)
      if (d[q] > 0) nuq[q][j] += R * d[q] / D;
  }
}

static void solve_cell(const ddo_ctx* c, int part, const cell_t* C, cell_out_t* o) {
  const lvl_t* l = &c->L[c->lev];
  const int s = c->s, nq = C->nq, nx = nq * s * s;
  const double cp = c->opt.cost_p, hp = pow(l->h, cp);
  const double eps = c->eps, lam = hp / eps;
  memset(o, 0, sizeof(*o));
  o->nq = nq;
  int32_t* ys = NULL;
  double* nuJ = NULL;
  int ny = cell_union(c, C, &ys, &nuJ);
  if (ny <= 0) {
    o->status = 2;
    free(ys);
    free(nuJ);
    return;
  }
  int *xr = malloc(sizeof(int) * nx), *xc = malloc(sizeof(int) * nx);
  int *yr = malloc(sizeof(int) * ny), *yc = malloc(sizeof(int) * ny);
  double *mu = malloc(sizeof(double) * nx), *F = malloc(sizeof(double) * nx);
  double *F0 = malloc(sizeof(double) * nx), *Fh = malloc(sizeof(double) * nx);
  double* G = malloc(sizeof(double) * ny);
  double* alpha = part == 0 ? c->aA : c->aB;
  double muJ = 0, mass_mu[4] = {0, 0, 0, 0};
  for (int k = 0; k < nx; k++) {
    cell_pixel(l, s, C, k, &xr[k], &xc[k]);
    int p = xr[k] * l->W + xc[k];
    mu[k] = l->mu[p];
    F[k] = alpha[p] / eps;
    F0[k] = F[k];
    muJ += mu[k];
    mass_mu[k / (s * s)] += mu[k];
  }
  for (int j = 0; j < ny; j++) {
    yr[j] = ys[j] / l->W;
    yc[j] = ys[j] % l->W;
  }
  double tol = c->opt.err_tol * muJ, err = 0;
  int loops = 0;
  int used = 0;
  /* A cell fails when it is not converged after the safeguard trigger (the
   * loop cap, or safeguard_after loops when that is set and smaller). */
  int cap0 = c->opt.max_iter;
  if (c->opt.safeguard && c->opt.safeguard_after > 0 && c->opt.safeguard_after < cap0)
    cap0 = c->opt.safeguard_after;
  int rc = sinkhorn_log(nx, xr, xc, mu, ny, yr, yc, nuJ, lam, cp, tol, cap0,
                        c->opt.accel, c->opt.newton_after, F, G, Fh, &loops, &err, &used);
  o->loops = loops;
  if (rc != 0 && c->opt.safeguard) {
    /* Safeguard of Sec. 7.4: solve the failing cell at a temporarily larger
     * eps (2 eps, same f), then return to eps from there.  READING: one
     * doubling, warm-started from the stored potential; each of the two
     * solves may take up to max_iter loops. */
    int l2 = 0, l3 = 0;
    for (int k = 0; k < nx; k++) F[k] = F0[k] * 0.5;
    int r2 = sinkhorn_log(nx, xr, xc, mu, ny, yr, yc, nuJ, lam * 0.5, cp, tol, c->opt.max_iter,
                          c->opt.accel, c->opt.newton_after, F, G, Fh, &l2, &err, &used);
    if (r2 != 2) {
      for (int k = 0; k < nx; k++) F[k] *= 2.0;
      rc = sinkhorn_log(nx, xr, xc, mu, ny, yr, yc, nuJ, lam, cp, tol, c->opt.max_iter,
                        c->opt.accel, c->opt.newton_after, F, G, Fh, &l3, &err, &used);
    } else {
      rc = 2;
    }
    o->loops += l2 + l3;
    o->status |= 4;
  }
  if (rc == 1) o->status |= 1;
  if (rc == 2) o->status |= 2;
  if (used) o->status |= 16;
  o->err = err;

  /* plan of the last Y-iteration, split into basic-cell Y-marginals
   * (Algorithm 2, "extract new basic partial marginals"), transport cost
   * <c,pi> and entropic objective eps*KL(pi|K) - eps*|K| written out from
   * the definition KL(pi|K) = sum pi log(pi/K) - pi + K, K = exp(-c/eps) mu nu */
  double* nuq[4];
  for (int q = 0; q < nq; q++) nuq[q] = calloc((size_t)ny, sizeof(double));
  double cost = 0, obj = 0;
  for (int k = 0; k < nx; k++) {
    if (!(mu[k] > 0)) continue;
    int q = k / (s * s);
    for (int j = 0; j < ny; j++) {
      double dr = xr[k] - yr[j], dc = xc[k] - yc[j];
      double cu = cost_units(dr, dc, cp);
      double e = F[k] + G[j] - lam * cu;
      double pi = exp(e) * mu[k] * nuJ[j];
      nuq[q][j] += pi;
      double cxy = hp * cu;
      cost += cxy * pi;
      if (pi > 0) {
        double nug = l->nu[ys[j]];
        obj += pi * (cxy + eps * (log(pi) - log(mu[k]) - log(nug)) - eps);
      }
    }
  }
  o->cost = cost;
  o->obj = obj;
  balance(nq, ny, nuq, mass_mu);
  /* Truncate (Sec. 6.1 (ii)): keep entries >= theta (and > 0). */
  for (int q = 0; q < nq; q++) {
    int n = 0;
    for (int j = 0; j < ny; j++)
      if (nuq[q][j] >= c->opt.trunc && nuq[q][j] > 0) n++;
    o->n[q] = n;
    o->col[q] = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    o->val[q] = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    n = 0;
    for (int j = 0; j < ny; j++)
      if (nuq[q][j] >= c->opt.trunc && nuq[q][j] > 0) {
        o->col[q][n] = ys[j];
        o->val[q][n] = nuq[q][j];
        n++;
      }
    free(nuq[q]);
  }
  /* store u_{C,J} as f = eps*F (Algorithm 2 output) */
  for (int k = 0; k < nx; k++) alpha[xr[k] * l->W + xc[k]] = eps * F[k];
  free(xr);
  free(xc);
  free(yr);
  free(yc);
  free(mu);
  free(F);
  free(F0);
  free(Fh);
  free(G);
  free(ys);
  free(nuJ);
}

/* ------------------------------------------------------------- lifecycle */

static int set_state_product(ddo_ctx* c) {
  /* Product coupling nu_i = |mu_i| nu, alpha = 0 (Sec. 6.4: the only
   * canonical feasible start without prior knowledge). */
  lvl_t* l = &c->L[c->lev];
  int s = c->s, npx = l->H * l->W;
  int nzy = 0;
  for (int p = 0; p < npx; p++)
    if (l->nu[p] > 0) nzy++;
  free(c->rp);
  free(c->col);
  free(c->val);
  c->rp = malloc(sizeof(int64_t) * (size_t)(c->nb + 1));
  c->col = malloc(sizeof(int32_t) * (size_t)c->nb * nzy);
  c->val = malloc(sizeof(double) * (size_t)c->nb * nzy);
  if (!c->rp || !c->col || !c->val) return -2;
  int64_t k = 0;
  for (int b = 0; b < c->nb; b++) {
    c->rp[b] = k;
    int br = b / l->bw, bc = b % l->bw;
    double m = 0;
    for (int a = 0; a < s; a++)
      for (int e = 0; e < s; e++) m += l->mu[(br * s + a) * l->W + bc * s + e];
    for (int p = 0; p < npx; p++)
      if (l->nu[p] > 0) {
        c->col[k] = p;
        c->val[k] = m * l->nu[p];
        k++;
      }
  }
  c->rp[c->nb] = k;
  free(c->aA);
  free(c->aB);
  c->aA = calloc((size_t)npx, sizeof(double));
  c->aB = calloc((size_t)npx, sizeof(double));
  return (c->aA && c->aB) ? 0 : -2;
}

void ddo_free(ddo_ctx* c) {
  if (!c) return;
  if (c->L)
    for (int i = 0; i < c->nlev; i++) {
      free(c->L[i].mu);
      free(c->L[i].nu);
    }
  free(c->L);
  free(c->rp);
  free(c->col);
  free(c->val);
  free(c->aA);
  free(c->aB);
  free(c->cells[0]);
  free(c->cells[1]);
  free(c->rc_cost);
  free(c->rc_obj);
  free(c->rc_err);
  free(c->rc_loops);
  free(c->rc_status);
  free(c);
}

int ddo_init(const double* mu, const double* nu, int H, int W, int s, int nlev, double eps,
             const ddo_opts* opt, ddo_ctx** out) {
  *out = NULL;
  if (!mu || !nu || H <= 0 || W <= 0 || s <= 0 || nlev < 1 || !(eps > 0) || !opt) return -1;
  int div = 2 * s << (nlev - 1);
  if (H % div || W % div) return -1;
  double sm = 0, sn = 0;
  for (int64_t p = 0; p < (int64_t)H * W; p++) {
    if (!(mu[p] >= 0) || !(nu[p] >= 0) || !isfinite(mu[p]) || !isfinite(nu[p])) return -1;
    sm += mu[p];
    sn += nu[p];
  }
  if (fabs(sm - 1) > 1e-9 || fabs(sn - 1) > 1e-9) return -1;
  if (!(opt->cost_p == 0 || opt->cost_p > 1) || opt->safeguard_after < 0) return -1;
  ddo_ctx* c = calloc(1, sizeof(ddo_ctx));
  if (!c) return -2;
  c->nlev = nlev;
  c->s = s;
  c->opt = *opt;
  if (c->opt.cost_p == 0) c->opt.cost_p = 2.0;
  c->eps = eps;
  c->L = calloc((size_t)nlev, sizeof(lvl_t));
  int mx = H > W ? H : W;
  for (int i = nlev - 1; i >= 0; i--) {
    lvl_t* l = &c->L[i];
    int f = nlev - 1 - i;
    l->H = H >> f;
    l->W = W >> f;
    l->bh = l->H / s;
    l->bw = l->W / s;
    l->h = (double)(1 << f) / mx;
    size_t n = (size_t)l->H * l->W;
    l->mu = malloc(sizeof(double) * n);
    l->nu = malloc(sizeof(double) * n);
    if (!l->mu || !l->nu) {
      ddo_free(c);
      return -2;
    }
    if (i == nlev - 1) {
      memcpy(l->mu, mu, sizeof(double) * n);
      memcpy(l->nu, nu, sizeof(double) * n);
    } else {
      /* coarse measure = push-forward under the parent map (Sec. 6.4) */
      lvl_t* fl = &c->L[i + 1];
      for (int r = 0; r < l->H; r++)
        for (int cc = 0; cc < l->W; cc++) {
          double a = 0, b = 0;
          for (int u = 0; u < 2; u++)
            for (int v = 0; v < 2; v++) {
              a += fl->mu[(2 * r + u) * fl->W + 2 * cc + v];
              b += fl->nu[(2 * r + u) * fl->W + 2 * cc + v];
            }
          l->mu[r * l->W + cc] = a;
          l->nu[r * l->W + cc] = b;
        }
    }
  }
  /* basic cells need positive mass (Definition of basic partitions) */
  lvl_t* fl = &c->L[nlev - 1];
  for (int b = 0; b < fl->bh * fl->bw; b++) {
    int br = b / fl->bw, bc = b % fl->bw;
    double m = 0;
    for (int a = 0; a < s; a++)
      for (int e = 0; e < s; e++) m += fl->mu[(br * s + a) * fl->W + bc * s + e];
    if (!(m > 0)) {
      ddo_free(c);
      return -1;
    }
  }
  c->lev = 0;
  c->last_part = -1;
  int rc = rebuild_cells(c);
  if (!rc) rc = set_state_product(c);
  if (rc) {
    ddo_free(c);
    return rc;
  }
  *out = c;
  return 0;
}

int ddo_set_eps(ddo_ctx* c, double eps) {
  /* f = eps*log u is kept fixed across an eps change (end of Sec. 6.4) */
  if (!c || !(eps > 0)) return -1;
  c->eps = eps;
  return 0;
}

int ddo_half_iterate(ddo_ctx* c, int part, const uint8_t* mask, ddo_iter_stats* st) {
  if (!c || (part != 0 && part != 1)) return -1;
  int nc = c->nc[part];
  const cell_t* cells = c->cells[part];
  cell_out_t* outs = calloc((size_t)nc, sizeof(cell_out_t));
  if (!outs) return -2;
#ifdef _OPENMP
  if (c->opt.n_threads > 0) omp_set_num_threads(c->opt.n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int k = 0; k < nc; k++) {
    const cell_t* C = &cells[k];
    if (mask && !mask[k]) {
      /* unselected cell: rows stay as they are */
      cell_out_t* o = &outs[k];
      o->nq = C->nq;
      o->status = 8;
      for (int q = 0; q < C->nq; q++) {
        int b = C->q[q];
        int64_t a = c->rp[b], n = c->rp[b + 1] - a;
        o->n[q] = (int)n;
        o->col[q] = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        o->val[q] = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        memcpy(o->col[q], c->col + a, sizeof(int32_t) * (size_t)n);
        memcpy(o->val[q], c->val + a, sizeof(double) * (size_t)n);
      }
    } else {
      solve_cell(c, part, C, &outs[k]);
    }
  }
  /* assemble the new basic-cell marginals in basic-cell order */
  int64_t* len = calloc((size_t)c->nb, sizeof(int64_t));
  for (int k = 0; k < nc; k++)
    for (int q = 0; q < cells[k].nq; q++) len[cells[k].q[q]] = outs[k].n[q];
  int64_t* rp = malloc(sizeof(int64_t) * (size_t)(c->nb + 1));
  rp[0] = 0;
  for (int b = 0; b < c->nb; b++) rp[b + 1] = rp[b] + len[b];
  int64_t nnz = rp[c->nb];
  int32_t* col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double* val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  ddo_iter_stats S;
  memset(&S, 0, sizeof(S));
  free(c->rc_cost);
  free(c->rc_obj);
  free(c->rc_err);
  free(c->rc_loops);
  free(c->rc_status);
  c->rc_cost = malloc(sizeof(double) * nc);
  c->rc_obj = malloc(sizeof(double) * nc);
  c->rc_err = malloc(sizeof(double) * nc);
  c->rc_loops = malloc(sizeof(int) * nc);
  c->rc_status = malloc(sizeof(int) * nc);
  c->rc_n = nc;
  for (int k = 0; k < nc; k++) {
    cell_out_t* o = &outs[k];
    for (int q = 0; q < cells[k].nq; q++) {
      int b = cells[k].q[q];
      memcpy(col + rp[b], o->col[q], sizeof(int32_t) * (size_t)o->n[q]);
      memcpy(val + rp[b], o->val[q], sizeof(double) * (size_t)o->n[q]);
      free(o->col[q]);
      free(o->val[q]);
    }
    c->rc_cost[k] = o->cost;
    c->rc_obj[k] = o->obj;
    c->rc_err[k] = o->err;
    c->rc_loops[k] = o->loops;
    c->rc_status[k] = o->status;
    if (o->status & 8) continue;
    S.n_cells++;
    S.loops_total += o->loops;
    if (o->loops > S.loops_max) S.loops_max = o->loops;
    if (o->status & 3) S.n_failed++;
    if (o->status & 4) S.n_safeguard++;
    if (o->status & 16) S.n_newton++;
    S.cost += o->cost;
    S.obj += o->obj;
    S.err_x += o->err;
  }
  S.nnz = nnz;
  free(c->rp);
  free(c->col);
  free(c->val);
  c->rp = rp;
  c->col = col;
  c->val = val;
  c->last_part = part;
  free(len);
  free(outs);
  if (st) *st = S;
  return S.n_failed ? 1 : 0;
}

/* ------------------------------------------------------------ refinement */

/* Conjugate gradients for the least-squares gluing potential V on the cells
 * of partition A:  min sum_e (V[b_e] - V[a_e] - w_e)^2  (Sec. 6.3).
 * READING: the sign follows the path-product definition of the glued
 * scalings (u_hat_J = prod q * u_{A,J}), i.e. V(J2)-V(J1) ~ log q(J1,J2). */
static void glue_cg(int n, int ne, const int* ea, const int* eb, const double* w, double* V) {
  double *b = calloc(n, sizeof(double)), *r = malloc(sizeof(double) * n),
         *p = malloc(sizeof(double) * n), *Ap = malloc(sizeof(double) * n);
  for (int e = 0; e < ne; e++) {
    b[eb[e]] += w[e];
    b[ea[e]] -= w[e];
  }
  for (int i = 0; i < n; i++) {
    V[i] = 0;
    r[i] = b[i];
    p[i] = b[i];
  }
  double rr = 0, bb = 0;
  for (int i = 0; i < n; i++) rr += r[i] * r[i];
  bb = rr;
  for (int it = 0; it < 20 * n + 100 && rr > 1e-28 * bb && rr > 0; it++) {
    for (int i = 0; i < n; i++) Ap[i] = 0;
    for (int e = 0; e < ne; e++) {
      double d = p[eb[e]] - p[ea[e]];
      Ap[eb[e]] += d;
      Ap[ea[e]] -= d;
    }
    double pAp = 0;
    for (int i = 0; i < n; i++) pAp += p[i] * Ap[i];
    if (!(pAp > 0)) break;
    double a = rr / pAp, rr2 = 0;
    for (int i = 0; i < n; i++) {
      V[i] += a * p[i];
      r[i] -= a * Ap[i];
      rr2 += r[i] * r[i];
    }
    double beta = rr2 / rr;
    rr = rr2;
    for (int i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
  }
  double mean = 0;
  for (int i = 0; i < n; i++) mean += V[i];
  mean /= n;
  for (int i = 0; i < n; i++) V[i] -= mean;
  free(b);
  free(r);
  free(p);
  free(Ap);
}

/* log of the mu-weighted mean of exp(sign*(fa-fb)/eps) over basic cell b */
static double log_mean_ratio(const lvl_t* l, int s, int b, const double* fa, const double* fb,
                             double eps, double sign) {
  int br = b / l->bw, bc = b % l->bw;
  double m = -INFINITY, tot = 0;
  for (int a = 0; a < s; a++)
    for (int e = 0; e < s; e++) {
      int p = (br * s + a) * l->W + bc * s + e;
      if (l->mu[p] > 0) {
        double v = sign * (fa[p] - fb[p]) / eps;
        if (v > m) m = v;
      }
    }
  double acc = 0;
  for (int a = 0; a < s; a++)
    for (int e = 0; e < s; e++) {
      int p = (br * s + a) * l->W + bc * s + e;
      if (l->mu[p] > 0) {
        acc += l->mu[p] * exp(sign * (fa[p] - fb[p]) / eps - m);
        tot += l->mu[p];
      }
    }
  return m + log(acc / tot);
}

/* bilinear interpolation of a coarse field at the fine pixel centres, with
 * linear extrapolation at the border (fine pixel i sits at coarse index
 * i/2 - 1/4) */
static double interp1(int n, double t, int* i0) {
  int i = (int)floor(t);
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  *i0 = i;
  return t - i;
}

int ddo_refine(ddo_ctx* c) {
  if (!c || c->lev >= c->nlev - 1) return -5;
  const int s = c->s;
  lvl_t* cl = &c->L[c->lev];
  lvl_t* fl = &c->L[c->lev + 1];
  const double eps = c->eps;
  /* 1. glue the A-cell potentials with the help of the B-cell ones */
  int na = c->nc[0];
  int *cellA = malloc(sizeof(int) * c->nb);
  for (int k = 0; k < na; k++)
    for (int q = 0; q < c->cells[0][k].nq; q++) cellA[c->cells[0][k].q[q]] = k;
  int ne = 0, cap = 12 * c->nc[1] + 8;
  int *ea = malloc(sizeof(int) * cap), *eb = malloc(sizeof(int) * cap);
  double* w = malloc(sizeof(double) * cap);
  /* every ordered pair of basic cells of one B-cell gives an oriented edge
   * between their A-cells: the weight depends on the orientation, and the
   * least squares takes both (the same graph as the certificate, Sec. 6.3) */
  for (int k = 0; k < c->nc[1]; k++) {
    const cell_t* C = &c->cells[1][k];
    for (int q1 = 0; q1 < C->nq; q1++)
      for (int q2 = 0; q2 < C->nq; q2++) {
        if (q2 == q1) continue;
        int b1 = C->q[q1], b2 = C->q[q2];
        /* log q(J1,J2) = log fint_{b1} u_A/u_B + log fint_{b2} u_B/u_A */
        double lq = log_mean_ratio(cl, s, b1, c->aA, c->aB, eps, 1.0) +
                    log_mean_ratio(cl, s, b2, c->aA, c->aB, eps, -1.0);
        ea[ne] = cellA[b1];
        eb[ne] = cellA[b2];
        w[ne] = lq;
        ne++;
      }
  }
  double* V = malloc(sizeof(double) * na);
  glue_cg(na, ne, ea, eb, w, V);
  double* fg = malloc(sizeof(double) * (size_t)cl->H * cl->W);
  for (int p = 0; p < cl->H * cl->W; p++) {
    int b = (p / cl->W / s) * cl->bw + (p % cl->W) / s;
    fg[p] = c->aA[p] + eps * V[cellA[b]];
  }
  /* 2. interpolate the glued f to the fine grid */
  size_t nf = (size_t)fl->H * fl->W;
  double* fa = malloc(sizeof(double) * nf);
  for (int r = 0; r < fl->H; r++) {
    int r0;
    double tr = interp1(cl->H, r * 0.5 - 0.25, &r0);
    for (int cc = 0; cc < fl->W; cc++) {
      int c0;
      double tc = interp1(cl->W, cc * 0.5 - 0.25, &c0);
      double v00 = fg[r0 * cl->W + c0], v01 = fg[r0 * cl->W + c0 + 1];
      double v10 = fg[(r0 + 1) * cl->W + c0], v11 = fg[(r0 + 1) * cl->W + c0 + 1];
      fa[(size_t)r * fl->W + cc] =
          (1 - tr) * ((1 - tc) * v00 + tc * v01) + tr * ((1 - tc) * v10 + tc * v11);
    }
  }
  /* 3. fine basic marginals, eq. (FineBasicMarginals):
   *    nu_i(y) = nu(y) * nuhat_{Pa(i)}(pa(y)) / nuhat(pa(y)) * mu(X_i) / muhat(Xhat_{Pa(i)}) */
  int nbf = fl->bh * fl->bw;
  int64_t* rp = malloc(sizeof(int64_t) * (nbf + 1));
  rp[0] = 0;
  for (int b = 0; b < nbf; b++) {
    int P = (b / fl->bw / 2) * cl->bw + (b % fl->bw) / 2;
    int64_t n = 0;
    for (int64_t k = c->rp[P]; k < c->rp[P + 1]; k++) {
      int y = c->col[k], yr = y / cl->W, yc = y % cl->W;
      (void)yr;
      (void)yc;
      n += 4;
    }
    rp[b + 1] = rp[b] + n;
  }
  int64_t nnz = rp[nbf];
  int32_t* col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  double* val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
  for (int b = 0; b < nbf; b++) {
    int br = b / fl->bw, bc = b % fl->bw;
    int P = (br / 2) * cl->bw + bc / 2;
    double mi = 0, mP = 0;
    for (int a = 0; a < s; a++)
      for (int e = 0; e < s; e++) mi += fl->mu[(br * s + a) * fl->W + bc * s + e];
    int pr = P / cl->bw, pc = P % cl->bw;
    for (int a = 0; a < s; a++)
      for (int e = 0; e < s; e++) mP += cl->mu[(pr * s + a) * cl->W + pc * s + e];
    int64_t k0 = rp[b], n = 0;
    /* all four children of each coarse support point (children of zero mass
     * are dropped by the next truncation), then sort by fine index */
    for (int64_t k = c->rp[P]; k < c->rp[P + 1]; k++) {
      int y = c->col[k], yr = y / cl->W, yc = y % cl->W;
      double ratio = c->val[k] / cl->nu[y];
      for (int u = 0; u < 2; u++)
        for (int v = 0; v < 2; v++) {
          int yf = (2 * yr + u) * fl->W + 2 * yc + v;
          col[k0 + n] = yf;
          val[k0 + n] = fl->nu[yf] * ratio * (mi / mP);
          n++;
        }
    }
    /* insertion sort of the (col,val) pairs of this row */
    for (int64_t i = 1; i < n; i++) {
      int32_t kc = col[k0 + i];
      double kv = val[k0 + i];
      int64_t j = i - 1;
      while (j >= 0 && col[k0 + j] > kc) {
        col[k0 + j + 1] = col[k0 + j];
        val[k0 + j + 1] = val[k0 + j];
        j--;
      }
      col[k0 + j + 1] = kc;
      val[k0 + j + 1] = kv;
    }
  }
  free(c->rp);
  free(c->col);
  free(c->val);
  c->rp = rp;
  c->col = col;
  c->val = val;
  free(c->aA);
  free(c->aB);
  c->aA = fa;
  c->aB = malloc(sizeof(double) * nf);
  memcpy(c->aB, fa, sizeof(double) * nf);
  c->lev++;
  c->last_part = -1;
  free(cellA);
  free(ea);
  free(eb);
  free(w);
  free(V);
  free(fg);
  return rebuild_cells(c);
}

int ddo_run_schedule(ddo_ctx* c, const ddo_stage* st, int n, ddo_iter_stats* total) {
  if (!c || !st || n < 0) return -1;
  ddo_iter_stats T;
  memset(&T, 0, sizeof(T));
  int warn = 0;
  for (int i = 0; i < n; i++) {
    while (c->lev < st[i].level) {
      int rc = ddo_refine(c);
      if (rc) return rc;
    }
    if (st[i].level != c->lev) return -1;
    ddo_set_eps(c, st[i].eps);
    for (int k = 0; k < st[i].n_half; k++) {
      ddo_iter_stats S;
      int rc = ddo_half_iterate(c, k & 1, NULL, &S);
      if (rc < 0) return rc;
      if (rc > 0) warn = 1;
      T.n_cells += S.n_cells;
      T.loops_total += S.loops_total;
      if (S.loops_max > T.loops_max) T.loops_max = S.loops_max;
      T.n_failed += S.n_failed;
      T.n_safeguard += S.n_safeguard;
      T.n_newton += S.n_newton;
      T.nnz = S.nnz;
      T.cost = S.cost;
      T.obj = S.obj;
      T.err_x = S.err_x;
    }
  }
  if (total) *total = T;
  return warn;
}

int ddo_cost(ddo_ctx* c, ddo_cost_report* r) {
  if (!c || !r) return -1;
  lvl_t* l = &c->L[c->lev];
  memset(r, 0, sizeof(*r));
  int npx = l->H * l->W;
  double* ym = calloc((size_t)npx, sizeof(double));
  double drift = 0;
  for (int b = 0; b < c->nb; b++) {
    double m = 0, mm = 0;
    for (int64_t k = c->rp[b]; k < c->rp[b + 1]; k++) {
      ym[c->col[k]] += c->val[k];
      m += c->val[k];
    }
    int br = b / l->bw, bc = b % l->bw;
    for (int a = 0; a < c->s; a++)
      for (int e = 0; e < c->s; e++) mm += l->mu[(br * c->s + a) * l->W + bc * c->s + e];
    drift += fabs(m - mm);
  }
  double ey = 0;
  for (int p = 0; p < npx; p++) ey += fabs(ym[p] - l->nu[p]);
  free(ym);
  r->err_y = ey;
  r->mass_drift = drift;
  r->nnz = c->rp[c->nb];
  r->level = c->lev;
  r->eps = c->eps;
  r->last_partition = c->last_part;
  if (c->last_part >= 0) {
    for (int k = 0; k < c->rc_n; k++) {
      r->cost += c->rc_cost[k];
      r->obj += c->rc_obj[k];
      r->err_x += c->rc_err[k];
    }
  }
  return 0;
}

int ddo_level_info(const ddo_ctx* c, int* level, int* H, int* W, int* n_basic, int* na,
                   int* nbb, double* eps, double* h) {
  if (!c) return -1;
  const lvl_t* l = &c->L[c->lev];
  if (level) *level = c->lev;
  if (H) *H = l->H;
  if (W) *W = l->W;
  if (n_basic) *n_basic = c->nb;
  if (na) *na = c->nc[0];
  if (nbb) *nbb = c->nc[1];
  if (eps) *eps = c->eps;
  if (h) *h = l->h;
  return 0;
}

int ddo_cells(const ddo_ctx* c, int part, int* cells) {
  if (!c || (part != 0 && part != 1) || !cells) return -1;
  for (int k = 0; k < c->nc[part]; k++)
    for (int q = 0; q < 4; q++) cells[k * 4 + q] = c->cells[part][k].q[q];
  return 0;
}

int ddo_export(const ddo_ctx* c, int64_t* nnz, int64_t* rp, int32_t* col, double* val,
               double* aA, double* aB) {
  if (!c) return -1;
  int64_t n = c->rp[c->nb];
  if (nnz) *nnz = n;
  const lvl_t* l = &c->L[c->lev];
  if (rp) memcpy(rp, c->rp, sizeof(int64_t) * (size_t)(c->nb + 1));
  if (col) memcpy(col, c->col, sizeof(int32_t) * (size_t)n);
  if (val) memcpy(val, c->val, sizeof(double) * (size_t)n);
  if (aA) memcpy(aA, c->aA, sizeof(double) * (size_t)l->H * l->W);
  if (aB) memcpy(aB, c->aB, sizeof(double) * (size_t)l->H * l->W);
  return 0;
}

int ddo_import(ddo_ctx* c, int level, double eps, const int64_t* rp, const int32_t* col,
               const double* val, const double* aA, const double* aB) {
  if (!c || level < 0 || level >= c->nlev || !(eps > 0) || !rp || !aA || !aB) return -1;
  c->lev = level;
  c->eps = eps;
  int rc = rebuild_cells(c);
  if (rc) return rc;
  const lvl_t* l = &c->L[level];
  int64_t n = rp[c->nb];
  free(c->rp);
  free(c->col);
  free(c->val);
  free(c->aA);
  free(c->aB);
  c->rp = malloc(sizeof(int64_t) * (size_t)(c->nb + 1));
  c->col = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  c->val = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  c->aA = malloc(sizeof(double) * (size_t)l->H * l->W);
  c->aB = malloc(sizeof(double) * (size_t)l->H * l->W);
  memcpy(c->rp, rp, sizeof(int64_t) * (size_t)(c->nb + 1));
  if (n) {
    memcpy(c->col, col, sizeof(int32_t) * (size_t)n);
    memcpy(c->val, val, sizeof(double) * (size_t)n);
  }
  memcpy(c->aA, aA, sizeof(double) * (size_t)l->H * l->W);
  memcpy(c->aB, aB, sizeof(double) * (size_t)l->H * l->W);
  c->last_part = -1;
  return 0;
}

int ddo_cell_results(const ddo_ctx* c, double* cost, double* obj, double* err, int* loops,
                     int* status) {
  if (!c || c->last_part < 0) return -5;
  for (int k = 0; k < c->rc_n; k++) {
    if (cost) cost[k] = c->rc_cost[k];
    if (obj) obj[k] = c->rc_obj[k];
    if (err) err[k] = c->rc_err[k];
    if (loops) loops[k] = c->rc_loops[k];
    if (status) status[k] = c->rc_status[k];
  }
  return 0;
}

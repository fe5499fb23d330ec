// Single sparse multi-scale Sinkhorn on the whole grid: the comparison method
// of Sec. 7.4 ("Comparison to single Sinkhorn algorithm"), a global Sinkhorn
// with absorbed (stabilised) potentials, adaptive kernel truncation, a
// coarse-to-fine scheme and eps-scaling.
//
// State of a level: absorbed potentials alpha(x), beta(y) (FP64, absolute
// units) and scalings u(x), v(y) relative to them; the plan is
//   pi(x,y) = u(x) v(y) exp((alpha(x) + beta(y) - c(x,y)) / eps) mu(x) nu(y)
// on the support S = {(x,y) : exp((alpha + beta - c)/eps) >= theta}, fixed
// between absorptions (the truncation of the stabilised kernel, Sec. 7.4).
// S is not stored: each x keeps the bounding box of its Y-points in S, each
// y the bounding box of its X-points, and every pass recomputes the kernel
// entries inside the box and tests membership with the same FP64 expression,
// so the X- and the Y-pass see exactly the same matrix.
//
// One thread per pixel.  FP64 exponents and sums, FP32 exponentials.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dd_internal.h"

namespace ddk {

namespace {

// exponent (alpha(x) + beta(y) - c(x,y)) / eps in one fixed order of FP64
// operations, shared by every kernel of this file
__device__ __forceinline__ double sg_exponent(double ax, double by, int dr, int dc, double hp,
                                              double half_p, double inv_eps) {
  return (ax + by - hp * cost_units(dr, dc, half_p)) * inv_eps;
}

constexpr int kSgThreads = 256;
constexpr int kSgMaxGrow = 64;  // window enlargements of one box search

// Bounding box of the points q of the other grid (H x W) with
// exponent(p, q) >= log_theta, searched in the candidate window `win`
// (inclusive rows r0..r1, cols c0..c1), enlarged by `margin` on every side
// where a kept point touches the window's edge (unless the edge is the
// grid's).  Writes the box (r0 > r1 if empty) and the number of kept points.
// DIR 0: p is an X pixel, q runs over Y; DIR 1: the reverse.
template <int DIR>
__global__ __launch_bounds__(kSgThreads) void k_sg_support(
    const double* pot_p, const double* pot_q, int H, int W, double hp, double half_p,
    double inv_eps, double log_theta, int margin, int4* box, long long* counts) {
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (p >= (long long)H * W) return;
  const int pr = (int)(p / W), pc = (int)(p % W);
  const double ap = pot_p[p];
  int4 w = box[p];  // candidate window
  w.x = max(w.x, 0);
  w.y = min(w.y, H - 1);
  w.z = max(w.z, 0);
  w.w = min(w.w, W - 1);
  int4 kept = make_int4(H, -1, W, -1);
  long long n = 0;
  for (int grow = 0; grow <= kSgMaxGrow; grow++) {
    kept = make_int4(H, -1, W, -1);
    n = 0;
    for (int r = w.x; r <= w.y; r++)
      for (int c = w.z; c <= w.w; c++) {
        const double e = DIR == 0 ? sg_exponent(ap, pot_q[(long long)r * W + c], pr - r, pc - c,
                                                hp, half_p, inv_eps)
                                  : sg_exponent(pot_q[(long long)r * W + c], ap, r - pr, c - pc,
                                                hp, half_p, inv_eps);
        if (e >= log_theta) {
          kept.x = min(kept.x, r);
          kept.y = max(kept.y, r);
          kept.z = min(kept.z, c);
          kept.w = max(kept.w, c);
          n++;
        }
      }
    if (n == 0 && (w.x > 0 || w.y < H - 1 || w.z > 0 || w.w < W - 1)) {
      w = make_int4(max(w.x - margin, 0), min(w.y + margin, H - 1), max(w.z - margin, 0),
                    min(w.w + margin, W - 1));
      continue;
    }
    bool grown = false;
    if (n > 0) {
      if (kept.x == w.x && w.x > 0) { w.x = max(w.x - margin, 0); grown = true; }
      if (kept.y == w.y && w.y < H - 1) { w.y = min(w.y + margin, H - 1); grown = true; }
      if (kept.z == w.z && w.z > 0) { w.z = max(w.z - margin, 0); grown = true; }
      if (kept.w == w.w && w.w < W - 1) { w.w = min(w.w + margin, W - 1); grown = true; }
    }
    if (!grown) break;
  }
  box[p] = kept;
  counts[p] = n;
}

__device__ double sg_block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
#pragma unroll
  for (int k = 0; k < kSgThreads / 64; k++) t += red[k];
  __syncthreads();
  return t;
}

__device__ double sg_block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = -INFINITY;
#pragma unroll
  for (int k = 0; k < kSgThreads / 64; k++) t = fmax(t, red[k]);
  __syncthreads();
  return t;
}

// One half of a Sinkhorn loop.  For every pixel p of this side:
//   s(p) = sum over q in S_p of exp(exponent) * scale_q(q) * m_q(q),
// the marginal of the current plan there is m_p(p) scale_p(p) s(p); with
// UPDATE the scaling becomes 1 / s(p) (the exact half-iteration).  Per block:
// part[0] = sum m_p |scale_p s - 1| (L1 error of the marginal), part[1] =
// max m_p |scale_p s - 1| (L-infinity error of the marginal), part[2] =
// max |log scale_p| after the update, part[3] = empty rows of positive mass,
// part[4] = kernel entries evaluated.
template <int DIR>
__global__ __launch_bounds__(kSgThreads) void k_sg_pass(
    const double* pot_p, const double* pot_q, const double* m_p, const double* m_q,
    double* scale_p, const double* scale_q, const int4* box, int H, int W, double hp,
    double half_p, double inv_eps, double log_theta, int update, double* part) {
  __shared__ double red[kSgThreads / 64];
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double l1 = 0, linf = 0, lmax = 0, empty = 0, evals = 0;
  if (p < (long long)H * W) {
    const int pr = (int)(p / W), pc = (int)(p % W);
    const double ap = pot_p[p];
    const int4 b = box[p];
    double s = 0;
    for (int r = b.x; r <= b.y; r++)
      for (int c = b.z; c <= b.w; c++) {
        const long long q = (long long)r * W + c;
        const double e = DIR == 0 ? sg_exponent(ap, pot_q[q], pr - r, pc - c, hp, half_p, inv_eps)
                                  : sg_exponent(pot_q[q], ap, r - pr, c - pc, hp, half_p, inv_eps);
        if (e >= log_theta) s += (double)__expf((float)e) * scale_q[q] * m_q[q];
      }
    if (b.y >= b.x && b.w >= b.z) evals = (double)(b.y - b.x + 1) * (double)(b.w - b.z + 1);
    const double mp = m_p[p];
    if (mp > 0) {
      if (!(s > 0)) {
        empty = 1;
      } else {
        const double d = scale_p[p] * s - 1.0;
        l1 = mp * fabs(d);
        linf = mp * fabs(d);
        if (update) {
          const double nsc = 1.0 / s;
          scale_p[p] = nsc;
          lmax = fabs(log(nsc));
        } else {
          lmax = fabs(log(scale_p[p]));
        }
      }
    }
  }
  l1 = sg_block_sum(l1, red);
  evals = sg_block_sum(evals, red);
  empty = sg_block_sum(empty, red);
  linf = sg_block_max(linf, red);
  lmax = sg_block_max(lmax, red);
  if (threadIdx.x == 0) {
    double* o = part + 5 * (size_t)blockIdx.x;
    o[0] = l1;
    o[1] = linf;
    o[2] = lmax;
    o[3] = empty;
    o[4] = evals;
  }
}

// Fixed-order reduction of the per-block partials: out[0..4] as above.
__global__ void k_sg_reduce(const double* part, int nblk, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double l1 = 0, linf = 0, lmax = 0, empty = 0, evals = 0;
  for (int k = 0; k < nblk; k++) {
    l1 += part[5 * k];
    linf = fmax(linf, part[5 * k + 1]);
    lmax = fmax(lmax, part[5 * k + 2]);
    empty += part[5 * k + 3];
    evals += part[5 * k + 4];
  }
  out[0] = l1;
  out[1] = linf;
  out[2] = lmax;
  out[3] = empty;
  out[4] = evals;
}

// Absorption: pot += eps log scale, scale = 1 (pixels of zero mass keep pot).
__global__ void k_sg_absorb(double* pot, double* scale, const double* m, long long n, double eps) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (m[i] > 0 && scale[i] > 0) pot[i] += eps * log(scale[i]);
  scale[i] = 1.0;
}

__global__ void k_sg_fill_box(int4* box, long long n, int4 v) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) box[i] = v;
}

__global__ void k_sg_fill(double* a, long long n, double v) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// Candidate windows after an eps change or an absorption: the current box
// enlarged by `margin` (an empty box becomes the whole grid).
__global__ void k_sg_widen(int4* box, long long n, int H, int W, int margin) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int4 b = box[i];
  if (b.y < b.x || b.w < b.z)
    b = make_int4(0, H - 1, 0, W - 1);
  else
    b = make_int4(b.x - margin, b.y + margin, b.z - margin, b.w + margin);
  box[i] = b;
}

// Candidate windows of the fine level: the children of the parent pixel's box
// on the coarse grid, enlarged by `margin` fine pixels.
__global__ void k_sg_refine_box(const int4* cbox, int Wc, int4* fbox, int Hf, int Wf,
                                int margin) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)Hf * Wf) return;
  const int r = (int)(i / Wf), c = (int)(i % Wf);
  int4 b = cbox[(long long)(r / 2) * Wc + c / 2];
  if (b.y < b.x || b.w < b.z)
    b = make_int4(0, Hf - 1, 0, Wf - 1);
  else
    b = make_int4(2 * b.x - margin, 2 * b.y + 1 + margin, 2 * b.z - margin, 2 * b.w + 1 + margin);
  fbox[i] = b;
}

// Plan sums over S after a Y-half (v up to date): per block part[0] =
// <c, pi>, part[1] = sum pi (log(pi / (mu nu)) + c/eps) - pi (the primal
// score KL(pi|K) - |K|), part[2] = sum pi; with the X-side view of S.
__global__ __launch_bounds__(kSgThreads) void k_sg_plan_sums(
    const double* alpha, const double* beta, const double* mu, const double* nu,
    const double* u, const double* v, const int4* box, int H, int W, double hp, double half_p,
    double eps, double log_theta, double* part) {
  __shared__ double red[kSgThreads / 64];
  const long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const double inv_eps = 1.0 / eps;
  double cost = 0, prim = 0, mass = 0;
  if (p < (long long)H * W && mu[p] > 0) {
    const int pr = (int)(p / W), pc = (int)(p % W);
    const double ap = alpha[p];
    const int4 b = box[p];
    for (int r = b.x; r <= b.y; r++)
      for (int c = b.z; c <= b.w; c++) {
        const long long q = (long long)r * W + c;
        const double e = sg_exponent(ap, beta[q], pr - r, pc - c, hp, half_p, inv_eps);
        if (!(e >= log_theta) || !(nu[q] > 0)) continue;
        const double lp = e + log(u[p]) + log(v[q]);  // log(pi / (mu nu))
        const double pi = exp(lp) * mu[p] * nu[q];
        const double cxy = hp * cost_units(pr - r, pc - c, half_p);
        cost += pi * cxy;
        prim += pi * (lp + cxy * inv_eps) - pi;
        mass += pi;
      }
  }
  cost = sg_block_sum(cost, red);
  prim = sg_block_sum(prim, red);
  mass = sg_block_sum(mass, red);
  if (threadIdx.x == 0) {
    part[3 * (size_t)blockIdx.x] = cost;
    part[3 * (size_t)blockIdx.x + 1] = prim;
    part[3 * (size_t)blockIdx.x + 2] = mass;
  }
}

// <alpha + eps log u, mu> and <beta + eps log v, nu> per block (the dual).
__global__ __launch_bounds__(kSgThreads) void k_sg_dual_sums(
    const double* alpha, const double* beta, const double* mu, const double* nu, const double* u,
    const double* v, long long n, double eps, double* part) {
  __shared__ double red[kSgThreads / 64];
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double a = 0, b = 0;
  if (i < n) {
    if (mu[i] > 0) a = (alpha[i] + eps * log(u[i])) * mu[i];
    if (nu[i] > 0) b = (beta[i] + eps * log(v[i])) * nu[i];
  }
  a = sg_block_sum(a, red);
  b = sg_block_sum(b, red);
  if (threadIdx.x == 0) {
    part[2 * (size_t)blockIdx.x] = a;
    part[2 * (size_t)blockIdx.x + 1] = b;
  }
}

__global__ void k_sg_reduce_n(const double* part, int nblk, int width, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int k = 0; k < width; k++) {
    double s = 0;
    for (int b = 0; b < nblk; b++) s += part[(size_t)width * b + k];
    out[k] = s;
  }
}

// Total potentials alpha + eps log u (the exported dual variables).
__global__ void k_sg_total(const double* pot, const double* scale, const double* m, long long n,
                           double eps, double* out) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = m[i] > 0 ? pot[i] + eps * log(scale[i]) : pot[i];
}

inline unsigned sg_blocks(long long n) { return (unsigned)((n + kSgThreads - 1) / kSgThreads); }

}  // namespace

void sg_launch_support(int dir, const double* pot_p, const double* pot_q, int H, int W,
                       double hp, double half_p, double eps, double log_theta, int margin,
                       int4* box, long long* counts, hipStream_t st) {
  const long long n = (long long)H * W;
  if (dir == 0)
    hipLaunchKernelGGL(k_sg_support<0>, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, pot_p, pot_q,
                       H, W, hp, half_p, 1.0 / eps, log_theta, margin, box, counts);
  else
    hipLaunchKernelGGL(k_sg_support<1>, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, pot_p, pot_q,
                       H, W, hp, half_p, 1.0 / eps, log_theta, margin, box, counts);
}

int sg_pass_blocks(int H, int W) { return (int)sg_blocks((long long)H * W); }

void sg_launch_pass(int dir, const double* pot_p, const double* pot_q, const double* m_p,
                    const double* m_q, double* scale_p, const double* scale_q, const int4* box,
                    int H, int W, double hp, double half_p, double eps, double log_theta,
                    int update, double* part, double* out5, hipStream_t st) {
  const long long n = (long long)H * W;
  const unsigned nb = sg_blocks(n);
  if (dir == 0)
    hipLaunchKernelGGL(k_sg_pass<0>, dim3(nb), dim3(kSgThreads), 0, st, pot_p, pot_q, m_p, m_q,
                       scale_p, scale_q, box, H, W, hp, half_p, 1.0 / eps, log_theta, update,
                       part);
  else
    hipLaunchKernelGGL(k_sg_pass<1>, dim3(nb), dim3(kSgThreads), 0, st, pot_p, pot_q, m_p, m_q,
                       scale_p, scale_q, box, H, W, hp, half_p, 1.0 / eps, log_theta, update,
                       part);
  if (out5) hipLaunchKernelGGL(k_sg_reduce, dim3(1), dim3(64), 0, st, part, (int)nb, out5);
}

void sg_launch_absorb(double* pot, double* scale, const double* m, long long n, double eps,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_sg_absorb, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, pot, scale, m, n,
                     eps);
}

void sg_launch_fill_box(int4* box, long long n, int4 v, hipStream_t st) {
  hipLaunchKernelGGL(k_sg_fill_box, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, box, n, v);
}

void sg_launch_fill(double* a, long long n, double v, hipStream_t st) {
  hipLaunchKernelGGL(k_sg_fill, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, a, n, v);
}

void sg_launch_widen(int4* box, long long n, int H, int W, int margin, hipStream_t st) {
  hipLaunchKernelGGL(k_sg_widen, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, box, n, H, W,
                     margin);
}

void sg_launch_refine_box(const int4* cbox, int Wc, int4* fbox, int Hf, int Wf, int margin,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_sg_refine_box, dim3(sg_blocks((long long)Hf * Wf)), dim3(kSgThreads), 0,
                     st, cbox, Wc, fbox, Hf, Wf, margin);
}

void sg_launch_final(const double* alpha, const double* beta, const double* mu, const double* nu,
                     const double* u, const double* v, const int4* xbox, int H, int W, double hp,
                     double half_p, double eps, double log_theta, double* part, double* out5,
                     hipStream_t st) {
  const long long n = (long long)H * W;
  const unsigned nb = sg_blocks(n);
  hipLaunchKernelGGL(k_sg_plan_sums, dim3(nb), dim3(kSgThreads), 0, st, alpha, beta, mu, nu, u, v,
                     xbox, H, W, hp, half_p, eps, log_theta, part);
  hipLaunchKernelGGL(k_sg_reduce_n, dim3(1), dim3(64), 0, st, part, (int)nb, 3, out5);
  hipLaunchKernelGGL(k_sg_dual_sums, dim3(nb), dim3(kSgThreads), 0, st, alpha, beta, mu, nu, u, v,
                     n, eps, part);
  hipLaunchKernelGGL(k_sg_reduce_n, dim3(1), dim3(64), 0, st, part, (int)nb, 2, out5 + 3);
}

void sg_launch_total(const double* pot, const double* scale, const double* m, long long n,
                     double eps, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sg_total, dim3(sg_blocks(n)), dim3(kSgThreads), 0, st, pot, scale, m, n,
                     eps, out);
}

}  // namespace ddk

// ---- host driver (C-ABI in include/dd_single.h) -------------------------

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dd_single.h"

namespace {

template <typename T>
hipError_t sg_alloc(T** p, size_t n) {
  *p = nullptr;
  return hipMalloc((void**)p, sizeof(T) * (n ? n : 1));
}

thread_local std::string g_sg_error;

dd_status sg_fail(dd_status s, const char* what) {
  g_sg_error = what;
  return s;
}

__global__ void k_sg_sum_counts(const long long* c, long long n, unsigned long long* out) {
  __shared__ unsigned long long sh;
  if (threadIdx.x == 0) sh = 0;
  __syncthreads();
  unsigned long long loc = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    loc += (unsigned long long)c[i];
  atomicAdd(&sh, loc);
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, sh);
}

struct SgLevel {
  int H = 0, W = 0;
  double h = 0;
  double* mu = nullptr;
  double* nu = nullptr;
};

}  // namespace

extern "C" void dd_single_options_default(dd_single_options* o) {
  if (!o) return;
  o->err_tol = 1e-7;
  o->err_norm = DD_SINGLE_LINF;
  o->theta = 1e-10;
  o->absorb = 30.0;
  o->max_iter = 200000;
  o->check_every = 16;
  o->cost_p = 2.0;
  o->stream = nullptr;
}

extern "C" const char* dd_single_last_error(void) { return g_sg_error.c_str(); }

extern "C" dd_status dd_single_solve(const double* mu_h, const double* nu_h, int H, int W,
                                     int nlev, const dd_stage* sched, int n_stages,
                                     const dd_single_options* opt_in, dd_single_report* rep,
                                     double* alpha_out, double* beta_out) {
  if (!mu_h || !nu_h || !sched || !rep || n_stages < 1 || nlev < 1 || nlev > 16 || H < 1 ||
      W < 1)
    return sg_fail(DD_EINVAL, "invalid arguments");
  dd_single_options opt;
  dd_single_options_default(&opt);
  if (opt_in) opt = *opt_in;
  if (!(opt.err_tol > 0) || !(opt.theta > 0 && opt.theta < 1) || !(opt.absorb > 0) ||
      opt.max_iter < 1 || opt.check_every < 1 || !(opt.cost_p > 1 && opt.cost_p <= 16))
    return sg_fail(DD_EINVAL, "invalid options");
  if ((H % (1 << (nlev - 1))) || (W % (1 << (nlev - 1))))
    return sg_fail(DD_EINVAL, "H and W must be divisible by 2^(n_levels-1)");
  for (int i = 0; i < n_stages; i++)
    if (!(sched[i].eps > 0) || sched[i].level < 0 || sched[i].level >= nlev ||
        (i > 0 && sched[i].level < sched[i - 1].level))
      return sg_fail(DD_EINVAL, "invalid schedule");
  const size_t nf = (size_t)H * W;
  double sm = 0, sn = 0;
  for (size_t i = 0; i < nf; i++) {
    if (!(mu_h[i] >= 0) || !(nu_h[i] >= 0) || !std::isfinite(mu_h[i]) || !std::isfinite(nu_h[i]))
      return sg_fail(DD_EINVAL, "negative or non-finite mass");
    sm += mu_h[i];
    sn += nu_h[i];
  }
  if (std::fabs(sm - 1) > 1e-9 || std::fabs(sn - 1) > 1e-9)
    return sg_fail(DD_EINVAL, "masses must sum to 1");
  hipStream_t st = (hipStream_t)opt.stream;
  const double half_p = 0.5 * opt.cost_p;
  const double log_theta = std::log(opt.theta);
  const int margin = 2;

  std::vector<SgLevel> L(nlev);
  std::vector<void*> owned;
  auto release = [&]() {
    for (void* p : owned) (void)hipFree(p);
    owned.clear();
  };
  hipError_t e = hipSuccess;
  auto alloc = [&](auto** p, size_t n) {
    if (e == hipSuccess) e = sg_alloc(p, n);
    if (e == hipSuccess) owned.push_back((void*)*p);
  };
  const int mx = std::max(H, W);
  for (int i = nlev - 1; i >= 0; i--) {
    SgLevel& l = L[i];
    const int f = nlev - 1 - i;
    l.H = H >> f;
    l.W = W >> f;
    l.h = (double)(1 << f) / mx;
    alloc(&l.mu, (size_t)l.H * l.W);
    alloc(&l.nu, (size_t)l.H * l.W);
  }
  double *alpha = nullptr, *beta = nullptr, *u = nullptr, *v = nullptr, *tmp = nullptr,
         *tmp2 = nullptr, *part = nullptr, *dout = nullptr, *hout = nullptr;
  int4 *xbox = nullptr, *ybox = nullptr, *cbox = nullptr;
  long long* counts = nullptr;
  unsigned long long* dsum = nullptr;
  alloc(&alpha, nf);
  alloc(&beta, nf);
  alloc(&u, nf);
  alloc(&v, nf);
  alloc(&tmp, nf);
  alloc(&tmp2, nf);
  alloc(&xbox, nf);
  alloc(&ybox, nf);
  alloc(&cbox, nf);
  alloc(&counts, nf);
  alloc(&part, 5 * (size_t)ddk::sg_pass_blocks(H, W) + 8);
  alloc(&dout, 16);
  alloc(&dsum, 2);
  if (e == hipSuccess) e = hipHostMalloc((void**)&hout, sizeof(double) * 16);
  if (e != hipSuccess) {
    release();
    if (hout) (void)hipHostFree(hout);
    return sg_fail(DD_ENOMEM, "allocation failed");
  }
  auto cleanup = [&]() {
    release();
    (void)hipHostFree(hout);
  };
  const auto t0 = std::chrono::steady_clock::now();
  e = hipMemcpyAsync(L[nlev - 1].mu, mu_h, sizeof(double) * nf, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(L[nlev - 1].nu, nu_h, sizeof(double) * nf, hipMemcpyHostToDevice, st);
  for (int i = nlev - 2; i >= 0 && e == hipSuccess; i--) {
    ddk::launch_pyramid(L[i + 1].mu, L[i].mu, L[i].H, L[i].W, st);
    ddk::launch_pyramid(L[i + 1].nu, L[i].nu, L[i].H, L[i].W, st);
  }
  memset(rep, 0, sizeof(*rep));
  int lev = 0;
  double eps = sched[0].eps;
  {
    const SgLevel& l = L[0];
    const long long n = (long long)l.H * l.W;
    ddk::sg_launch_fill(alpha, n, 0.0, st);
    ddk::sg_launch_fill(beta, n, 0.0, st);
    ddk::sg_launch_fill(u, n, 1.0, st);
    ddk::sg_launch_fill(v, n, 1.0, st);
    ddk::sg_launch_fill_box(xbox, n, make_int4(0, l.H - 1, 0, l.W - 1), st);
    ddk::sg_launch_fill_box(ybox, n, make_int4(0, l.H - 1, 0, l.W - 1), st);
  }
  auto read = [&](int k) -> hipError_t {
    hipError_t r = hipMemcpyAsync(hout, dout, sizeof(double) * k, hipMemcpyDeviceToHost, st);
    if (r == hipSuccess) r = hipStreamSynchronize(st);
    return r;
  };
  // the support of both sides from the current potentials at eps, and its size
  auto support = [&](const SgLevel& l, double hp) -> hipError_t {
    const long long n = (long long)l.H * l.W;
    ddk::sg_launch_support(0, alpha, beta, l.H, l.W, hp, half_p, eps, log_theta, margin, xbox,
                           counts, st);
    hipError_t r = hipMemsetAsync(dsum, 0, sizeof(unsigned long long), st);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL(k_sg_sum_counts, dim3(256), dim3(256), 0, st, counts, n, dsum);
    ddk::sg_launch_support(1, beta, alpha, l.H, l.W, hp, half_p, eps, log_theta, margin, ybox,
                           counts, st);
    unsigned long long hs = 0;
    r = hipMemcpyAsync(&hs, dsum, sizeof hs, hipMemcpyDeviceToHost, st);
    if (r == hipSuccess) r = hipStreamSynchronize(st);
    rep->entries_final = (int64_t)hs;
    rep->entries_max = std::max(rep->entries_max, (int64_t)hs);
    return r;
  };
  bool failed = false;
  for (int si = 0; si < n_stages && e == hipSuccess && !failed; si++) {
    const dd_stage& sg = sched[si];
    while (lev < sg.level && e == hipSuccess) {
      // refinement: total potentials interpolated to the fine pixels (the
      // same bilinear rule as the decomposition's refinement), boxes from
      // the parents' boxes, scalings reset
      const SgLevel& lc = L[lev];
      const SgLevel& lfn = L[lev + 1];
      const long long ncs = (long long)lc.H * lc.W, nfs = (long long)lfn.H * lfn.W;
      ddk::sg_launch_total(alpha, u, lc.mu, ncs, eps, tmp, st);
      ddk::launch_interp(tmp, lc.H, lc.W, alpha, tmp2, lfn.H, lfn.W, st);
      ddk::sg_launch_total(beta, v, lc.nu, ncs, eps, tmp, st);
      ddk::launch_interp(tmp, lc.H, lc.W, beta, tmp2, lfn.H, lfn.W, st);
      e = hipMemcpyAsync(cbox, xbox, sizeof(int4) * ncs, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) break;
      ddk::sg_launch_refine_box(cbox, lc.W, xbox, lfn.H, lfn.W, margin, st);
      e = hipMemcpyAsync(cbox, ybox, sizeof(int4) * ncs, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) break;
      ddk::sg_launch_refine_box(cbox, lc.W, ybox, lfn.H, lfn.W, margin, st);
      ddk::sg_launch_fill(u, nfs, 1.0, st);
      ddk::sg_launch_fill(v, nfs, 1.0, st);
      lev++;
    }
    if (e != hipSuccess) break;
    const SgLevel& l = L[lev];
    const long long n = (long long)l.H * l.W;
    const double hp = std::pow(l.h, opt.cost_p);
    // eps change: potentials in absolute units stay (absorbed at the old eps)
    ddk::sg_launch_absorb(alpha, u, l.mu, n, eps, st);
    ddk::sg_launch_absorb(beta, v, l.nu, n, eps, st);
    eps = sg.eps;
    if (si > 0) {
      ddk::sg_launch_widen(xbox, n, l.H, l.W, margin, st);
      ddk::sg_launch_widen(ybox, n, l.H, l.W, margin, st);
    }
    e = support(l, hp);
    if (e != hipSuccess) break;
    int it = 0, last_check = 0;
    bool done = false;
    while (!done && e == hipSuccess) {
      it++;
      const bool check = (it % opt.check_every) == 0 || it >= opt.max_iter;
      // Y-half (exact): v = 1 / column sums
      ddk::sg_launch_pass(1, beta, alpha, l.nu, l.mu, v, u, ybox, l.H, l.W, hp, half_p, eps,
                          log_theta, 1, part, check ? dout + 5 : nullptr, st);
      if (check) {
        // X-marginal error of the plan after the Y-half
        ddk::sg_launch_pass(0, alpha, beta, l.mu, l.nu, u, v, xbox, l.H, l.W, hp, half_p, eps,
                            log_theta, 0, part, dout, st);
        e = read(10);
        if (e != hipSuccess) break;
        // kernel entries evaluated by the loops since the last check (box
        // areas of both passes) and by this check's extra X-pass
        rep->entry_evals += (int64_t)((hout[4] + hout[9]) * (it - last_check) + hout[4]);
        last_check = it;
        const double err = opt.err_norm == DD_SINGLE_L1 ? hout[0] : hout[1];
        if (hout[3] > 0 || hout[8] > 0 || !std::isfinite(err)) {
          failed = true;  // a row or column of positive mass lost its whole support
          break;
        }
        if (err <= opt.err_tol) {
          rep->err_x_l1 = hout[0];
          rep->err_x_linf = hout[1];
          done = true;
          break;
        }
        if (it >= opt.max_iter) {
          rep->err_x_l1 = hout[0];
          rep->err_x_linf = hout[1];
          failed = true;
          break;
        }
        if (hout[2] > opt.absorb || hout[7] > opt.absorb) {
          ddk::sg_launch_absorb(alpha, u, l.mu, n, eps, st);
          ddk::sg_launch_absorb(beta, v, l.nu, n, eps, st);
          ddk::sg_launch_widen(xbox, n, l.H, l.W, margin, st);
          ddk::sg_launch_widen(ybox, n, l.H, l.W, margin, st);
          e = support(l, hp);
          rep->n_absorb++;
          if (e != hipSuccess) break;
        }
      }
      // X-half: u = 1 / row sums
      ddk::sg_launch_pass(0, alpha, beta, l.mu, l.nu, u, v, xbox, l.H, l.W, hp, half_p, eps,
                          log_theta, 1, part, nullptr, st);
    }
    rep->loops_total += it;
    rep->loops_max_stage = std::max(rep->loops_max_stage, it);
    rep->n_stages++;
  }
  if (e == hipSuccess && !failed) {
    const SgLevel& l = L[lev];
    const long long n = (long long)l.H * l.W;
    const double hp = std::pow(l.h, opt.cost_p);
    // Y-marginal error of the final plan (exact up to rounding after a Y-half)
    ddk::sg_launch_pass(1, beta, alpha, l.nu, l.mu, v, u, ybox, l.H, l.W, hp, half_p, eps,
                        log_theta, 0, part, dout, st);
    e = read(5);
    if (e == hipSuccess) rep->err_y_l1 = hout[0];
    if (e == hipSuccess) {
      ddk::sg_launch_final(alpha, beta, l.mu, l.nu, u, v, xbox, l.H, l.W, hp, half_p, eps,
                           log_theta, part, dout, st);
      e = read(5);
    }
    if (e == hipSuccess) {
      rep->cost = hout[0];
      rep->primal = hout[1];  // already in units of the KL divergence
      rep->dual = (hout[3] + hout[4]) / eps - hout[2];
      rep->plan_mass = hout[2];
    }
    if (e == hipSuccess && alpha_out) {
      ddk::sg_launch_total(alpha, u, l.mu, n, eps, tmp, st);
      e = hipMemcpyAsync(alpha_out, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e == hipSuccess && beta_out) {
      ddk::sg_launch_total(beta, v, l.nu, n, eps, tmp, st);
      e = hipMemcpyAsync(beta_out, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  rep->ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  rep->level = lev;
  rep->eps = eps;
  cleanup();
  if (e != hipSuccess) return sg_fail(DD_EHIP, hipGetErrorString(e));
  if (failed) {
    rep->failed = 1;
    g_sg_error = "a stage hit the iteration cap or a row or column lost its support";
    return DD_ENOTCONV;
  }
  return DD_OK;
}

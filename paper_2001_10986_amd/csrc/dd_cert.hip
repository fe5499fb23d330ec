// Kernels of the primal-dual certificate (Sec. 6.3, "Estimating the primal-dual
// gap"): the exact Y-iteration of the glued X-potential over the support of
// the stored plan, and the FP64 sums of the dual objective J
// (eq. EntropicOTDualObjective).  Not part of a sweep; FP64 throughout.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dd_internal.h"

namespace ddk {

namespace {

// Order-preserving map of doubles onto unsigned 64-bit keys (for atomicMax).
__device__ inline unsigned long long dkey(double v) {
  unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double dunkey(unsigned long long k) {
  unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

__global__ void k_cert_fill(unsigned long long* M, double* S, long long npx, double* sums) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < npx) {
    M[i] = dkey(-INFINITY);
    S[i] = 0.0;
  }
  if (i < 4) sums[i] = 0.0;
}

// One wavefront per basic cell; its lanes walk the cell's stored Y-support.
// pass 0: M(y) = max over x in X_i of (alpha_hat(x) - c(x,y))/eps + log mu(x);
// pass 1: S(y) += sum over x in X_i of exp(that - M(y)).
template <int PASS>
__global__ void k_cert_y(const int64_t* row_off, const int* row_len, const int* col,
                         const double* alpha_hat, const double* mu, int bs, int W, int bw,
                         int n_basic,
                         double inv_eps, double hp, double half_p, unsigned long long* M,
                         double* S) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int n_waves = (gridDim.x * blockDim.x) >> 6;
  for (int b = wave; b < n_basic; b += n_waves) {
    const int br = b / bw, bc = b % bw;
    const int64_t off = row_off[b];
    const int len = row_len[b];
    for (int e = lane; e < len; e += 64) {
      const int y = col[off + e];
      const int yr = y / W, yc = y % W;
      const double m = PASS == 1 ? dunkey(M[y]) : 0.0;
      double acc = PASS == 0 ? -INFINITY : 0.0;
      for (int i = 0; i < bs; i++)
        for (int j = 0; j < bs; j++) {
          const int xr = br * bs + i, xc = bc * bs + j;
          const long long px = (long long)xr * W + xc;
          const double mx = mu[px];
          if (!(mx > 0)) continue;
          const double t =
              (alpha_hat[px] - hp * cost_units(xr - yr, xc - yc, half_p)) * inv_eps + log(mx);
          if (PASS == 0)
            acc = t > acc ? t : acc;
          else
            acc += exp(t - m);
        }
      if (PASS == 0)
        atomicMax(&M[y], dkey(acc));
      else
        atomicAdd(&S[y], acc);
    }
  }
}

// sums[0] = sum alpha_hat mu, sums[1] = sum beta_hat nu, sums[2] = sum nu,
// sums[3] = number of pixels with nu > 0 that no stored entry reaches.
__global__ void k_cert_sums(const double* alpha_hat, const double* mu, const double* nu,
                            const unsigned long long* M, const double* S, long long npx,
                            double eps, double* beta_hat, double* sums) {
  __shared__ double red[4][256];
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < npx;
       i += (long long)gridDim.x * blockDim.x) {
    s0 += alpha_hat[i] * mu[i];
    const double n = nu[i];
    double b = NAN;
    if (S[i] > 0) {
      b = -eps * (dunkey(M[i]) + log(S[i]));
      if (n > 0) s1 += b * n;
    } else if (n > 0) {
      s3 += 1.0;
    }
    beta_hat[i] = b;
    s2 += n;
  }
  red[0][threadIdx.x] = s0;
  red[1][threadIdx.x] = s1;
  red[2][threadIdx.x] = s2;
  red[3][threadIdx.x] = s3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; k++) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) atomicAdd(&sums[threadIdx.x], red[threadIdx.x][0]);
}

// Right-hand side of the normal equations of the gluing least squares:
// rhs(J) = sum of log q over the oriented edges ending at J minus the sum over
// those starting at J; inc_e holds (edge << 1) | (J is the edge's head).
__global__ void k_cert_rhs(const int* inc_ptr, const int* inc_e, const int* e_ia,
                           const int* e_ib, const double* q, int na, double* rhs) {
  const int J = blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= na) return;
  double s = 0;
  for (int k = inc_ptr[J]; k < inc_ptr[J + 1]; k++) {
    const int e = inc_e[k] >> 1;
    const double w = q[2 * e_ia[e]] + q[2 * e_ib[e] + 1];
    s += (inc_e[k] & 1) ? w : -w;
  }
  rhs[J] = s;
}

constexpr int kCgThreads = 1024;

// Workgroup sum in a fixed order: a butterfly over the 64 lanes of each wave
// (every lane ends with the wave's sum), one slot per wave in LDS, and every
// thread adds the 16 slots itself (two barriers).
__device__ double cg_reduce(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
#pragma unroll
  for (int w = 0; w < kCgThreads / 64; w++) t += red[w];
  __syncthreads();  // the slots are reused by the next reduction
  return t;
}

// Conjugate gradients for L V = rhs in one workgroup, L the graph Laplacian
// of the A-cell graph (deg on the diagonal, -w for each neighbour, the
// neighbour lists in ELL form with zero-weight padding); L is
// singular on constants and rhs sums to zero, so the iterates stay in the
// complement; V is shifted to mean zero at the end.  Each thread owns the
// rows J = tid + k*1024 of x, r and Ap; p is read across threads, through
// agent-scope loads after a release fence and the barrier.  The loop ends
// for all waves at the same step (every test reads workgroup-reduced values).
__global__ __launch_bounds__(kCgThreads) void k_cert_cg(
    const int* ell_idx, const double* ell_w, int ell_k, const double* deg,
    const double* b, int na, int max_it, double tol2, double* x, double* r, double* p,
    double* Ap, double* info) {
  __shared__ double red[kCgThreads / 64];
  const int tid = threadIdx.x;
  double loc = 0;
  for (int J = tid; J < na; J += kCgThreads) {
    x[J] = 0;
    r[J] = b[J];
    p[J] = b[J];
    loc += b[J] * b[J];
  }
  double rr = cg_reduce(loc, red);
  const double bb = rr;
  __threadfence();
  __syncthreads();
  __threadfence();
  int it = 0;
  while (it < max_it && rr > tol2 * bb && rr > 0) {
    loc = 0;
    for (int J = tid; J < na; J += kCgThreads) {
      double v = deg[J] * p[J];
      for (int k0 = 0; k0 < ell_k; k0 += 8) {
        int idx[8];
        double w[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
          idx[k] = ell_idx[(size_t)(k0 + k) * na + J];
          w[k] = ell_w[(size_t)(k0 + k) * na + J];
        }
#pragma unroll
        for (int k = 0; k < 8; k++)
          v -= w[k] * __hip_atomic_load(&p[idx[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      Ap[J] = v;
      loc += p[J] * v;
    }
    const double pAp = cg_reduce(loc, red);
    if (!(pAp > 0)) break;
    const double a = rr / pAp;
    loc = 0;
    for (int J = tid; J < na; J += kCgThreads) {
      x[J] += a * p[J];
      r[J] -= a * Ap[J];
      loc += r[J] * r[J];
    }
    const double rr2 = cg_reduce(loc, red);
    const double beta = rr2 / rr;
    rr = rr2;
    for (int J = tid; J < na; J += kCgThreads) p[J] = r[J] + beta * p[J];
    __threadfence();
    __syncthreads();
    __threadfence();
    it++;
  }
  loc = 0;
  for (int J = tid; J < na; J += kCgThreads) loc += x[J];
  const double mean = cg_reduce(loc, red) / (na > 0 ? na : 1);
  for (int J = tid; J < na; J += kCgThreads) x[J] -= mean;
  if (tid == 0) {
    info[0] = it;
    info[1] = rr;
    info[2] = bb;
  }
}

// The same iteration for na <= ROWS * kCgThreads with the search direction p
// in LDS (read by every thread in the Laplacian product) and x, r, Ap in
// registers: the same operations in the same order as k_cert_cg, so the same
// result, without the global-memory round trips of p on every step.
template <int ROWS>
__global__ __launch_bounds__(kCgThreads) void k_cert_cg_lds(
    const int* ell_idx, const double* ell_w, int ell_k, const double* deg,
    const double* b, int na, int max_it, double tol2, double* x_out, double* info) {
  __shared__ double red[kCgThreads / 64];
  __shared__ double ps[ROWS * kCgThreads];
  const int tid = threadIdx.x;
  double x[ROWS], r[ROWS], ap[ROWS];
  double loc = 0;
#pragma unroll
  for (int q = 0; q < ROWS; q++) {
    const int J = tid + q * kCgThreads;
    const double bj = J < na ? b[J] : 0.0;
    x[q] = 0;
    r[q] = bj;
    ap[q] = 0;
    ps[J] = bj;
    if (J < na) loc += bj * bj;
  }
  double rr = cg_reduce(loc, red);
  const double bb = rr;
  __syncthreads();
  int it = 0;
  while (it < max_it && rr > tol2 * bb && rr > 0) {
    loc = 0;
#pragma unroll
    for (int q = 0; q < ROWS; q++) {
      const int J = tid + q * kCgThreads;
      if (J < na) {
        double v = deg[J] * ps[J];
        for (int k0 = 0; k0 < ell_k; k0 += 8) {
          int idx[8];
          double w[8];
#pragma unroll
          for (int k = 0; k < 8; k++) {
            idx[k] = ell_idx[(size_t)(k0 + k) * na + J];
            w[k] = ell_w[(size_t)(k0 + k) * na + J];
          }
#pragma unroll
          for (int k = 0; k < 8; k++) v -= w[k] * ps[idx[k]];
        }
        ap[q] = v;
        loc += ps[J] * v;
      }
    }
    const double pAp = cg_reduce(loc, red);
    if (!(pAp > 0)) break;
    const double a = rr / pAp;
    loc = 0;
#pragma unroll
    for (int q = 0; q < ROWS; q++) {
      const int J = tid + q * kCgThreads;
      if (J < na) {
        x[q] += a * ps[J];
        r[q] -= a * ap[q];
        loc += r[q] * r[q];
      }
    }
    const double rr2 = cg_reduce(loc, red);
    const double beta = rr2 / rr;
    rr = rr2;
#pragma unroll
    for (int q = 0; q < ROWS; q++) {
      const int J = tid + q * kCgThreads;
      if (J < na) ps[J] = r[q] + beta * ps[J];
    }
    __syncthreads();
    it++;
  }
  loc = 0;
#pragma unroll
  for (int q = 0; q < ROWS; q++)
    if (tid + q * kCgThreads < na) loc += x[q];
  const double mean = cg_reduce(loc, red) / (na > 0 ? na : 1);
#pragma unroll
  for (int q = 0; q < ROWS; q++) {
    const int J = tid + q * kCgThreads;
    if (J < na) x_out[J] = x[q] - mean;
  }
  if (tid == 0) {
    info[0] = it;
    info[1] = rr;
    info[2] = bb;
  }
}

constexpr int kCgLdsRows = 4;  // p in LDS up to 4096 unknowns (32 KiB)

}  // namespace

void launch_cert_glue(const int* inc_ptr, const int* inc_e, const int* e_ia, const int* e_ib,
                      const double* q, const int* ell_idx, const double* ell_w, int ell_k,
                      const double* deg, int na, int max_it, double tol2, double* work,
                      double* V, double* info, hipStream_t st) {
  double* rhs = work;
  double* r = work + na;
  double* p = work + 2 * (size_t)na;
  double* Ap = work + 3 * (size_t)na;
  hipLaunchKernelGGL(k_cert_rhs, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, st, inc_ptr,
                     inc_e, e_ia, e_ib, q, na, rhs);
  if (na <= kCgLdsRows * kCgThreads)
    hipLaunchKernelGGL((k_cert_cg_lds<kCgLdsRows>), dim3(1), dim3(kCgThreads), 0, st, ell_idx,
                       ell_w, ell_k, deg, rhs, na, max_it, tol2, V, info);
  else
    hipLaunchKernelGGL(k_cert_cg, dim3(1), dim3(kCgThreads), 0, st, ell_idx, ell_w, ell_k, deg,
                       rhs, na, max_it, tol2, V, r, p, Ap, info);
}

void launch_cert_y(const int64_t* row_off, const int* row_len, const int* col,
                   const double* alpha_hat, const double* mu, const double* nu, int H, int W,
                   int bs, int bw, int n_basic, double eps, double h, double half_p,
                   double* scratch, double* beta_hat, double* sums, hipStream_t st) {
  const long long npx = (long long)H * W;
  unsigned long long* M = (unsigned long long*)scratch;
  double* S = scratch + npx;
  hipLaunchKernelGGL(k_cert_fill, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, st, M, S,
                     npx, sums);
  const unsigned blocks = (unsigned)((n_basic + 3) / 4 < 65535 ? (n_basic + 3) / 4 : 65535);
  hipLaunchKernelGGL(k_cert_y<0>, dim3(blocks), dim3(256), 0, st, row_off, row_len, col,
                     alpha_hat, mu, bs, W, bw, n_basic, 1.0 / eps, std::pow(h, 2.0 * half_p),
                     half_p, M, S);
  hipLaunchKernelGGL(k_cert_y<1>, dim3(blocks), dim3(256), 0, st, row_off, row_len, col,
                     alpha_hat, mu, bs, W, bw, n_basic, 1.0 / eps, std::pow(h, 2.0 * half_p),
                     half_p, M, S);
  hipLaunchKernelGGL(k_cert_sums, dim3(1024), dim3(256), 0, st, alpha_hat, mu, nu, M, S, npx,
                     eps, beta_hat, sums);
}

}  // namespace ddk

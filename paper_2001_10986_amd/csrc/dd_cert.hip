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
                         const double* alpha_hat, const double* mu, int W, int bw, int n_basic,
                         double inv_eps, double h2, unsigned long long* M, double* S) {
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
      for (int i = 0; i < kS; i++)
        for (int j = 0; j < kS; j++) {
          const int xr = br * kS + i, xc = bc * kS + j;
          const long long px = (long long)xr * W + xc;
          const double mx = mu[px];
          if (!(mx > 0)) continue;
          const double dr = xr - yr, dc = xc - yc;
          const double t = (alpha_hat[px] - h2 * (dr * dr + dc * dc)) * inv_eps + log(mx);
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

}  // namespace

void launch_cert_y(const int64_t* row_off, const int* row_len, const int* col,
                   const double* alpha_hat, const double* mu, const double* nu, int H, int W,
                   int bw, int n_basic, double eps, double h, double* scratch, double* beta_hat,
                   double* sums, hipStream_t st) {
  const long long npx = (long long)H * W;
  unsigned long long* M = (unsigned long long*)scratch;
  double* S = scratch + npx;
  hipLaunchKernelGGL(k_cert_fill, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, st, M, S,
                     npx, sums);
  const unsigned blocks = (unsigned)((n_basic + 3) / 4 < 65535 ? (n_basic + 3) / 4 : 65535);
  hipLaunchKernelGGL(k_cert_y<0>, dim3(blocks), dim3(256), 0, st, row_off, row_len, col,
                     alpha_hat, mu, W, bw, n_basic, 1.0 / eps, h * h, M, S);
  hipLaunchKernelGGL(k_cert_y<1>, dim3(blocks), dim3(256), 0, st, row_off, row_len, col,
                     alpha_hat, mu, W, bw, n_basic, 1.0 / eps, h * h, M, S);
  hipLaunchKernelGGL(k_cert_sums, dim3(1024), dim3(256), 0, st, alpha_hat, mu, nu, M, S, npx,
                     eps, beta_hat, sums);
}

}  // namespace ddk

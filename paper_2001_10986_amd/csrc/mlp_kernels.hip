// gfx950 kernels of the warm-start network: a 4-layer MLP (width 256) whose
// GEMMs run on BF16 matrix cores (v_mfma_f32_32x32x8bf16_1k) with FP32
// accumulation, its ReLU/bias epilogues, the masked MSE loss, the backward
// pass and Adam on FP32 master weights.  Used for inference inside a sweep
// (warm start of the cell solves) and for training on cell problems that the
// plain method generated.
#include "mlp_internal.h"

#include <math.h>

namespace mlpk {

typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // round to nearest even
}
__device__ __forceinline__ float bf16_float(unsigned short b) {
  return __uint_as_float((unsigned)b << 16);
}

// C[M x N] = A[M x K] B[K x N] (+ epilogue).  A(m,k) = a[m*lda + k] (or
// a[k*lda + m] when TA), B(k,n) = b[k*ldb + n] (or b[n*ldb + k] when TB), BF16.
// M, N multiples of 64, K multiple of 32 (callers pad).  A block computes one
// 64x64 tile with 4 waves, one 32x32 quadrant each; K advances by 32 through
// LDS, the tiles loaded along the contiguous index of each operand's layout.
// Matrix-core operand layout: lane l holds rows/cols (l%32) and k
// (4(l/32) .. +3); the result element (i, j) of register v is
// i = 8(v/4) + 4(l/32) + v%4, j = l%32.  Split K (gridDim.z > 1): block z
// takes K-range z of gridDim.z equal ones and writes its raw partial tile to
// part + z*M*N; k_splitk_reduce then sums the partials in order of z and
// applies the epilogue (the same result for every launch).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(const unsigned short* __restrict__ a, int lda,
                                              const unsigned short* __restrict__ b, int ldb,
                                              int M, int N, int K, Epilogue ep,
                                              float* __restrict__ part) {
  __shared__ unsigned short As[64][32 + 4];
  __shared__ unsigned short Bs[32][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int qi = wave >> 1, qj = wave & 1;
  const int kc = K / (int)gridDim.z;  // a multiple of 32 (checked by the launcher)
  const int kb = (int)blockIdx.z * kc, ke = kb + kc;
  floatx16 acc = {};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    for (int e = tid; e < 64 * 32; e += 256) {
      int r, k;  // A tile element (r, k), consecutive threads on contiguous addresses
      if (TA) { k = e >> 6; r = e & 63; } else { r = e >> 5; k = e & 31; }
      const int gm = m0 + r, gk = k0 + k;
      As[r][k] = TA ? a[(size_t)gk * lda + gm] : a[(size_t)gm * lda + gk];
    }
    for (int e = tid; e < 32 * 64; e += 256) {
      int k, c;  // B tile element (k, c)
      if (TB) { c = e >> 5; k = e & 31; } else { k = e >> 6; c = e & 63; }
      const int gk = k0 + k, gn = n0 + c;
      Bs[k][c] = TB ? b[(size_t)gn * ldb + gk] : b[(size_t)gk * ldb + gn];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 8) {
      short4_t av, bv;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        av[t] = (short)As[32 * qi + (lane & 31)][kk + 4 * (lane >> 5) + t];
        bv[t] = (short)Bs[kk + 4 * (lane >> 5) + t][32 * qj + (lane & 31)];
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  float* pz = gridDim.z > 1 ? part + (size_t)blockIdx.z * M * N : nullptr;
#pragma unroll
  for (int v = 0; v < 16; v++) {
    const int i = m0 + 32 * qi + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int j = n0 + 32 * qj + (lane & 31);
    float x = acc[v];
    const size_t at = (size_t)i * N + j;
    if (pz) {
      pz[at] = x;
      continue;
    }
    if (ep.bias) x += ep.bias[j];
    if (ep.out_f32) ep.out_f32[at] = x;             // pre-activation / plain output
    if (ep.relu) x = x > 0.f ? x : 0.f;
    if (ep.out_bf16) ep.out_bf16[at] = bf16_bits(x);  // next layer's input
    if (ep.accum_f32) ep.accum_f32[at] += x;         // gradient accumulation
  }
}

__global__ void k_splitk_reduce(const float* __restrict__ part, int nz, int M, int N,
                                Epilogue ep) {
  const size_t MN = (size_t)M * N;
  for (size_t at = (size_t)blockIdx.x * blockDim.x + threadIdx.x; at < MN;
       at += (size_t)gridDim.x * blockDim.x) {
    float x = 0.f;
    for (int z = 0; z < nz; z++) x += part[(size_t)z * MN + at];
    const int j = (int)(at % N);
    if (ep.bias) x += ep.bias[j];
    if (ep.out_f32) ep.out_f32[at] = x;
    if (ep.relu) x = x > 0.f ? x : 0.f;
    if (ep.out_bf16) ep.out_bf16[at] = bf16_bits(x);
    if (ep.accum_f32) ep.accum_f32[at] += x;
  }
}

int gemm_splits(int M, int N, int K) {
  // split K when the output has fewer tiles than compute units and K is long
  const int tiles = (M / 64) * (N / 64);
  int z = 1;
  while (z < kMaxSplitK && tiles * z < 256 && K % (64 * z) == 0 && K / (2 * z) >= 256) z *= 2;
  return z;
}

void launch_gemm(bool ta, bool tb, const unsigned short* a, int lda, const unsigned short* b,
                 int ldb, int M, int N, int K, const Epilogue& ep, float* part, hipStream_t st) {
  const int z = part ? gemm_splits(M, N, K) : 1;
  dim3 grid(N / 64, M / 64, z);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, a, lda, b, ldb, M, N, K, ep, part);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, a, lda, b, ldb, M, N, K, ep, part);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, a, lda, b, ldb, M, N, K, ep, part);
  else hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, a, lda, b, ldb, M, N, K, ep, part);
  if (z > 1) hipLaunchKernelGGL(k_splitk_reduce, dim3(256), dim3(256), 0, st, part, z, M, N, ep);
}

// FP32 -> BF16 copy of an n_rows x n_cols matrix into a zero-padded
// rows x ld buffer (rows >= n_rows, ld >= n_cols)
__global__ void k_to_bf16_pad(const float* __restrict__ x, int n_rows, int n_cols, int rows, int ld,
                              unsigned short* __restrict__ y) {
  const size_t n = (size_t)rows * ld;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / ld), c = (int)(e % ld);
    y[e] = (r < n_rows && c < n_cols) ? bf16_bits(x[(size_t)r * n_cols + c]) : (unsigned short)0;
  }
}
void launch_to_bf16_pad(const float* x, int n_rows, int n_cols, int rows, int ld,
                        unsigned short* y, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16_pad, dim3(512), dim3(256), 0, st, x, n_rows, n_cols, rows, ld, y);
}

// Masked MSE: L = sum mask (y - t)^2 / sum mask over the first n rows; the
// gradient dL/dy goes out in BF16 (rows beyond n and masked entries are 0).
// Partial sums per block, then a fixed-order final sum (deterministic).
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             const float* __restrict__ mask, int n, int rows,
                                             int d, const float* __restrict__ inv_count,
                                             unsigned short* __restrict__ g, float* part) {
  __shared__ float sh[256];
  float acc = 0.f;
  const size_t total = (size_t)rows * d;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / d);
    float gr = 0.f;
    if (r < n) {
      const float m = mask[e], diff = y[e] - t[e];
      acc += m * diff * diff;
      gr = 2.f * m * diff * inv_count[0];
    }
    g[e] = bf16_bits(gr);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
// 1 / sum(mask) over the first n rows (one block, fixed order)
// 1 / (number of masked entries); the mask holds 0/1, so the FP32 sum of
// fewer than 2^24 of them is exact in any order
__global__ __launch_bounds__(1024) void k_mask_count(const float* __restrict__ mask, size_t ne,
                                                     float* out) {
  __shared__ float sh[16];
  float acc = 0.f;
  const size_t n4 = ne / 4;
  const float4* m4 = reinterpret_cast<const float4*>(mask);
  for (size_t e = threadIdx.x; e < n4; e += 1024) {
    const float4 v = m4[e];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  for (size_t e = 4 * n4 + threadIdx.x; e < ne; e += 1024) acc += mask[e];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int w = 0; w < 16; w++) s += sh[w];
    out[0] = s > 0.f ? 1.f / s : 0.f;
  }
}
__global__ void k_sum_parts(const float* part, int n, const float* inv_count, float* out) {
  if (threadIdx.x == 0) {
    float s = 0.f;
    for (int k = 0; k < n; k++) s += part[k];
    out[0] = s * inv_count[0];
  }
}
void launch_mse(const float* y, const float* t, const float* mask, int n, int rows, int d,
                unsigned short* g, float* part, float* scal, hipStream_t st) {
  hipLaunchKernelGGL(k_mask_count, dim3(1), dim3(1024), 0, st, mask, (size_t)n * d, scal + 1);
  hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, st, y, t, mask, n, rows, d, scal + 1,
                     g, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, st, part, kMseBlocks, scal + 1, scal);
}

// dz = dh * [z > 0] in BF16, dh given in FP32
__global__ void k_relu_back(const float* __restrict__ dh, const float* __restrict__ z, size_t n,
                            unsigned short* __restrict__ dz) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    dz[e] = bf16_bits(z[e] > 0.f ? dh[e] : 0.f);
}
void launch_relu_back(const float* dh, const float* z, size_t n, unsigned short* dz,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_relu_back, dim3(512), dim3(256), 0, st, dh, z, n, dz);
}

// db[j] = sum_r g[r][j] (BF16 gradient rows): a block of 64 columns x 16
// row lanes (coalesced 128-byte row segments), each lane summing every 16th
// row, the 16 lane sums added in lane order
__global__ __launch_bounds__(1024) void k_bias_grad(const unsigned short* __restrict__ g, int rows,
                                                    int d, float* __restrict__ db) {
  __shared__ float sh[16][64];
  const int c = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  float s = 0.f;
  if (j < d)
    for (int r = rl; r < rows; r += 16) s += bf16_float(g[(size_t)r * d + j]);
  sh[rl][c] = s;
  __syncthreads();
  if (rl == 0 && j < d) {
    float t = 0.f;
    for (int k = 0; k < 16; k++) t += sh[k][c];
    db[j] = t;
  }
}
void launch_bias_grad(const unsigned short* g, int rows, int d, float* db, hipStream_t st) {
  hipLaunchKernelGGL(k_bias_grad, dim3((d + 63) / 64), dim3(1024), 0, st, g, rows, d, db);
}

// Adam on the FP32 master weights, then their BF16 copy
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, size_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, unsigned short* __restrict__ wb) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x) {
    const float gg = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * gg;
    const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
    m[e] = mm;
    v[e] = vv;
    const float x = w[e] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    w[e] = x;
    if (wb) wb[e] = bf16_bits(x);
  }
}
void launch_adam(float* w, const float* g, float* m, float* v, size_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, unsigned short* wb, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(512), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps, c1, c2, wb);
}

__global__ void k_f32_to_bf16(const float* __restrict__ x, size_t n, unsigned short* __restrict__ y) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = bf16_bits(x[e]);
}
void launch_f32_to_bf16(const float* x, size_t n, unsigned short* y, hipStream_t st) {
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(512), dim3(256), 0, st, x, n, y);
}

// copy the first n rows x d columns of an FP32 rows x d matrix
__global__ void k_copy_rows(const float* __restrict__ x, size_t n, float* __restrict__ y) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    y[e] = x[e];
}
void launch_copy(const float* x, size_t n, float* y, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_rows, dim3(512), dim3(256), 0, st, x, n, y);
}

}  // namespace mlpk

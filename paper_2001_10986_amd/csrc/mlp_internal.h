// Internal interface of the warm-start network kernels (mlp_kernels.hip) for
// its runtime (mlp_runtime.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mlpk {

// What the GEMM does with each result element x (after + bias when given):
// out_f32 = x; then ReLU if relu; out_bf16 = bf16(x); accum_f32 += x.
struct Epilogue {
  const float* bias;
  float* out_f32;
  unsigned short* out_bf16;
  float* accum_f32;
  int relu;
};

constexpr int kMseBlocks = 256;

constexpr int kMaxSplitK = 8;  // K splits of a GEMM at most (workspace: kMaxSplitK * M * N floats)
int gemm_splits(int M, int N, int K);
// part: split-K workspace of kMaxSplitK * M * N floats, or nullptr (no split)
void launch_gemm(bool ta, bool tb, const unsigned short* a, int lda, const unsigned short* b,
                 int ldb, int M, int N, int K, const Epilogue& ep, float* part, hipStream_t st);
void launch_to_bf16_pad(const float* x, int n_rows, int n_cols, int rows, int ld,
                        unsigned short* y, hipStream_t st);
void launch_mse(const float* y, const float* t, const float* mask, int n, int rows, int d,
                unsigned short* g, float* part, float* scal, hipStream_t st);
void launch_relu_back(const float* dh, const float* z, size_t n, unsigned short* dz,
                      hipStream_t st);
void launch_bias_grad(const unsigned short* g, int rows, int d, float* db, hipStream_t st);
void launch_adam(float* w, const float* g, float* m, float* v, size_t n, float lr, float b1,
                 float b2, float eps, float c1, float c2, unsigned short* wb, hipStream_t st);
void launch_f32_to_bf16(const float* x, size_t n, unsigned short* y, hipStream_t st);
void launch_copy(const float* x, size_t n, float* y, hipStream_t st);

}  // namespace mlpk

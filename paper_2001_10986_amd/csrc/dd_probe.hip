// Measured issue rates of the arithmetic the solvers are built from: FP32
// fused multiply-adds (not packed: packed FP32 is disabled in this build),
// FP64 fused multiply-adds and the FP32 exponential (v_exp_f32).  Each
// thread runs eight independent dependency chains for a fixed number of
// steps; the grid holds eight workgroups of four waves per compute unit, so
// every SIMD has eight waves to interleave.  The rate is the best of three
// timed launches after one warm-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/dd.h"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeChains = 8;
constexpr int kProbeBlocksPerCu = 8;
constexpr int kProbeReps = 3;

thread_local std::string g_probe_error;

// The chains stay finite (|b| < 1, small c).  The final sum is written only
// when it equals a value it never takes, which keeps every chain live
// without a store per thread.
__global__ __launch_bounds__(kProbeThreads) void k_probe_fma32(float b, float c, int steps,
                                                               float* out) {
  float a[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; i++) a[i] = 1e-3f * (float)threadIdx.x + (float)i;
  for (int t = 0; t < steps; t += 8) {
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int i = 0; i < kProbeChains; i++) a[i] = fmaf(a[i], b, c);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeChains; i++) s += a[i];
  if (s == -1234.5f) out[blockIdx.x] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_fma64(double b, double c, int steps,
                                                               double* out) {
  double a[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; i++) a[i] = 1e-3 * (double)threadIdx.x + (double)i;
  for (int t = 0; t < steps; t += 8) {
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int i = 0; i < kProbeChains; i++) a[i] = fma(a[i], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kProbeChains; i++) s += a[i];
  if (s == -1234.5) out[blockIdx.x] = s;
}

// x -> 2^(-x) maps [0, 8] into (0, 1] and converges, so the chains stay
// finite; the negation is a source modifier of v_exp_f32.
__global__ __launch_bounds__(kProbeThreads) void k_probe_exp32(int steps, float* out) {
  float a[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; i++) a[i] = 1e-3f * (float)threadIdx.x + (float)i;
  for (int t = 0; t < steps; t += 8) {
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int i = 0; i < kProbeChains; i++) a[i] = __builtin_amdgcn_exp2f(-a[i]);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kProbeChains; i++) s += a[i];
  if (s == -1234.5f) out[blockIdx.x] = s;
}

// Best time in ms of kProbeReps launches (after one warm-up) of `launch`.
template <class F>
hipError_t best_ms(hipStream_t st, F launch, float* best) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  *best = 1e30f;
  for (int r = 0; r < kProbeReps && e == hipSuccess; r++) {
    e = hipEventRecord(e0, st);
    if (e != hipSuccess) break;
    launch();
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) *best = std::min(*best, ms);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

}  // namespace

extern "C" dd_status dd_probe_peaks(dd_peaks* out) {
  if (!out) {
    g_probe_error = "null output";
    return DD_EINVAL;
  }
  *out = dd_peaks{};
  int dev = 0, cus = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev);
  if (e != hipSuccess || cus <= 0) {
    g_probe_error = std::string("device query failed: ") + hipGetErrorString(e);
    return DD_EHIP;
  }
  const int blocks = cus * kProbeBlocksPerCu;
  const double lanes = (double)blocks * kProbeThreads * kProbeChains;
  const int steps32 = 8192, steps64 = 4096, steps_exp = 2048;
  hipStream_t st = nullptr;
  void* buf = nullptr;
  e = hipStreamCreate(&st);
  if (e == hipSuccess) e = hipMalloc(&buf, sizeof(double) * (size_t)blocks);
  float ms32 = 0.f, ms64 = 0.f, msx = 0.f;
  if (e == hipSuccess)
    e = best_ms(st, [&] {
      hipLaunchKernelGGL(k_probe_fma32, dim3(blocks), dim3(kProbeThreads), 0, st, 0.9999f, 1e-4f,
                         steps32, (float*)buf);
    }, &ms32);
  if (e == hipSuccess)
    e = best_ms(st, [&] {
      hipLaunchKernelGGL(k_probe_fma64, dim3(blocks), dim3(kProbeThreads), 0, st, 0.9999, 1e-4,
                         steps64, (double*)buf);
    }, &ms64);
  if (e == hipSuccess)
    e = best_ms(st, [&] {
      hipLaunchKernelGGL(k_probe_exp32, dim3(blocks), dim3(kProbeThreads), 0, st, steps_exp,
                         (float*)buf);
    }, &msx);
  if (st) (void)hipStreamSynchronize(st);
  if (buf) (void)hipFree(buf);
  if (st) (void)hipStreamDestroy(st);
  if (e != hipSuccess) {
    g_probe_error = std::string("probe launch failed: ") + hipGetErrorString(e);
    return DD_EHIP;
  }
  out->fp32_fma_tflops = 2.0 * lanes * steps32 / (ms32 * 1e-3) * 1e-12;
  out->fp64_fma_tflops = 2.0 * lanes * steps64 / (ms64 * 1e-3) * 1e-12;
  out->exp_f32_per_s = lanes * steps_exp / (msx * 1e-3);
  out->compute_units = cus;
  out->clock_mhz = khz * 1e-3;
  out->ms_fp32 = ms32;
  out->ms_fp64 = ms64;
  out->ms_exp = msx;
  return DD_OK;
}

extern "C" const char* dd_probe_last_error(void) { return g_probe_error.c_str(); }

// Host side of the warm-start network: parameter storage, forward pass,
// masked-MSE gradients and Adam steps, all enqueued on the network's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "../../include/dd_mlp.h"
#include "mlp_internal.h"

struct dd_mlp {
  int n_in, n_out, width;
  int dims[5];           // n_in, width, width, width, n_out
  size_t off_w[4], off_b[4], n_params;
  hipStream_t st = nullptr;
  float* w = nullptr;    // FP32 master parameters (flat)
  float* g = nullptr;    // gradient (flat)
  float* m = nullptr;    // Adam moments
  float* v = nullptr;
  unsigned short* wb = nullptr;  // BF16 copy of the flat parameters (biases unused)
  int step = 0;
  // activations, sized for `rows` rows
  int rows = 0;
  unsigned short *xb = nullptr, *hb[3] = {}, *gy = nullptr, *dz = nullptr;
  float *z[3] = {}, *y = nullptr, *dh = nullptr;
  float* part = nullptr;
  float* ksplit = nullptr; // split-K partial tiles of the weight-gradient GEMMs
  float* scal = nullptr;   // [0] loss, [1] 1/count
  float* hscal = nullptr;  // pinned
  std::string err;
};

static dd_status mfail(dd_mlp* n, dd_status s, const char* msg) {
  if (n) n->err = msg;
  return s;
}
#define MCHK(n, call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess) return mfail(n, DD_EHIP, hipGetErrorString(e_));   \
  } while (0)

template <typename T>
static hipError_t dm(T** p, size_t n) {
  *p = nullptr;
  return hipMalloc((void**)p, sizeof(T) * (n ? n : 1));
}

// split-K workspace: the largest weight matrix, kMaxSplitK times
static size_t ksplit_floats(const int* d) {
  size_t mx = 0;
  for (int l = 0; l < 4; l++) mx = std::max(mx, (size_t)d[l] * d[l + 1]);
  return mx * mlpk::kMaxSplitK;
}

static void free_act(dd_mlp* n) {
  hipFree(n->xb);
  for (int i = 0; i < 3; i++) {
    hipFree(n->hb[i]);
    hipFree(n->z[i]);
    n->hb[i] = nullptr;
    n->z[i] = nullptr;
  }
  hipFree(n->gy);
  hipFree(n->dz);
  hipFree(n->y);
  hipFree(n->dh);
  n->xb = n->gy = n->dz = nullptr;
  n->y = n->dh = nullptr;
  n->rows = 0;
}

static dd_status ensure_rows(dd_mlp* n, int rows) {
  if (rows <= n->rows) return DD_OK;
  free_act(n);
  const int W = n->width;
  MCHK(n, dm(&n->xb, (size_t)rows * n->n_in));
  for (int i = 0; i < 3; i++) {
    MCHK(n, dm(&n->hb[i], (size_t)rows * W));
    MCHK(n, dm(&n->z[i], (size_t)rows * W));
  }
  MCHK(n, dm(&n->gy, (size_t)rows * n->n_out));
  MCHK(n, dm(&n->dz, (size_t)rows * W));
  MCHK(n, dm(&n->y, (size_t)rows * n->n_out));
  MCHK(n, dm(&n->dh, (size_t)rows * W));
  n->rows = rows;
  return DD_OK;
}

extern "C" dd_status dd_mlp_create(int n_in, int n_out, int width, unsigned long long seed,
                                   void* stream, dd_mlp** out) {
  if (!out) return DD_EINVAL;
  *out = nullptr;
  if (n_in <= 0 || n_in % 64 || n_out <= 0 || n_out % 64 || width <= 0 || width % 64)
    return DD_EINVAL;
  dd_mlp* n = new dd_mlp();
  n->n_in = n_in;
  n->n_out = n_out;
  n->width = width;
  const int d[5] = {n_in, width, width, width, n_out};
  size_t off = 0;
  for (int l = 0; l < 4; l++) {
    n->dims[l] = d[l];
    n->off_w[l] = off;
    off += (size_t)d[l] * d[l + 1];
    n->off_b[l] = off;
    off += d[l + 1];
  }
  n->dims[4] = d[4];
  n->n_params = off;
  n->st = (hipStream_t)stream;
  if (dm(&n->w, off) || dm(&n->g, off) || dm(&n->m, off) || dm(&n->v, off) || dm(&n->wb, off) ||
      dm(&n->part, mlpk::kMseBlocks) || dm(&n->scal, 4) || dm(&n->ksplit, ksplit_floats(d)) ||
      hipHostMalloc((void**)&n->hscal, sizeof(float) * 4) != hipSuccess) {
    dd_mlp_free(n);
    return DD_ENOMEM;
  }
  // He initialisation (normal, std sqrt(2/fan_in)), zero biases, from a fixed
  // seed; the output layer starts 10x smaller (a near-zero initial output)
  std::vector<float> h(off, 0.f);
  std::mt19937_64 rng(seed);
  for (int l = 0; l < 4; l++) {
    std::normal_distribution<float> nd(0.f, std::sqrt(2.f / d[l]) * (l == 3 ? 0.1f : 1.f));
    for (size_t k = 0; k < (size_t)d[l] * d[l + 1]; k++) h[n->off_w[l] + k] = nd(rng);
  }
  dd_status s = dd_mlp_set_params(n, h.data(), off);
  if (s) {
    dd_mlp_free(n);
    return s;
  }
  *out = n;
  return DD_OK;
}

extern "C" void dd_mlp_free(dd_mlp* n) {
  if (!n) return;
  if (n->st) hipStreamSynchronize(n->st);
  else hipDeviceSynchronize();
  free_act(n);
  hipFree(n->w);
  hipFree(n->g);
  hipFree(n->m);
  hipFree(n->v);
  hipFree(n->wb);
  hipFree(n->part);
  hipFree(n->ksplit);
  hipFree(n->scal);
  if (n->hscal) hipHostFree(n->hscal);
  delete n;
}

extern "C" const char* dd_mlp_last_error(const dd_mlp* n) { return n ? n->err.c_str() : ""; }

extern "C" void* dd_mlp_get_stream(const dd_mlp* n) { return n ? (void*)n->st : nullptr; }

extern "C" dd_status dd_mlp_shape(const dd_mlp* n, int* n_in, int* n_out, int* width,
                                  size_t* n_params) {
  if (!n) return DD_EINVAL;
  if (n_in) *n_in = n->n_in;
  if (n_out) *n_out = n->n_out;
  if (width) *width = n->width;
  if (n_params) *n_params = n->n_params;
  return DD_OK;
}

extern "C" dd_status dd_mlp_set_params(dd_mlp* n, const float* host, size_t count) {
  if (!n || !host || count != n->n_params) return DD_EINVAL;
  MCHK(n, hipMemcpyAsync(n->w, host, sizeof(float) * count, hipMemcpyHostToDevice, n->st));
  MCHK(n, hipMemsetAsync(n->m, 0, sizeof(float) * count, n->st));
  MCHK(n, hipMemsetAsync(n->v, 0, sizeof(float) * count, n->st));
  mlpk::launch_f32_to_bf16(n->w, count, n->wb, n->st);
  MCHK(n, hipGetLastError());
  MCHK(n, hipStreamSynchronize(n->st));
  n->step = 0;
  return DD_OK;
}

extern "C" dd_status dd_mlp_get_params(const dd_mlp* n, float* host, size_t count) {
  if (!n || !host || count != n->n_params) return DD_EINVAL;
  dd_mlp* nn = const_cast<dd_mlp*>(n);
  MCHK(nn, hipMemcpyAsync(host, n->w, sizeof(float) * count, hipMemcpyDeviceToHost, n->st));
  MCHK(nn, hipStreamSynchronize(n->st));
  return DD_OK;
}

// forward on R = rows padded to 64; x already in n->xb
static void forward_padded(dd_mlp* n, int R) {
  const unsigned short* in = n->xb;
  for (int l = 0; l < 4; l++) {
    mlpk::Epilogue ep{};
    ep.bias = n->w + n->off_b[l];
    if (l < 3) {
      ep.out_f32 = n->z[l];
      ep.relu = 1;
      ep.out_bf16 = n->hb[l];
    } else {
      ep.out_f32 = n->y;
    }
    mlpk::launch_gemm(false, false, in, n->dims[l], n->wb + n->off_w[l], n->dims[l + 1], R,
                      n->dims[l + 1], n->dims[l], ep, nullptr, n->st);
    if (l < 3) in = n->hb[l];
  }
}

extern "C" dd_status dd_mlp_forward_bf16(dd_mlp* n, const unsigned short* xb_dev, int n_rows,
                                         float* y_dev) {
  if (!n || n_rows < 0 || (n_rows > 0 && (!xb_dev || !y_dev))) return DD_EINVAL;
  if (n_rows == 0) return DD_OK;
  if (n_rows % 64) return mfail(n, DD_EINVAL, "rows of a BF16 batch must be a multiple of 64");
  dd_status s = ensure_rows(n, n_rows);
  if (s) return s;
  MCHK(n, hipMemcpyAsync(n->xb, xb_dev, sizeof(unsigned short) * (size_t)n_rows * n->n_in,
                         hipMemcpyDeviceToDevice, n->st));
  forward_padded(n, n_rows);
  mlpk::launch_copy(n->y, (size_t)n_rows * n->n_out, y_dev, n->st);
  MCHK(n, hipGetLastError());
  return DD_OK;
}

extern "C" dd_status dd_mlp_forward(dd_mlp* n, const float* x_dev, int n_rows, float* y_dev) {
  if (!n || n_rows < 0 || (n_rows > 0 && (!x_dev || !y_dev))) return DD_EINVAL;
  if (n_rows == 0) return DD_OK;
  const int R = (n_rows + 63) / 64 * 64;
  dd_status s = ensure_rows(n, R);
  if (s) return s;
  mlpk::launch_to_bf16_pad(x_dev, n_rows, n->n_in, R, n->n_in, n->xb, n->st);
  forward_padded(n, R);
  mlpk::launch_copy(n->y, (size_t)n_rows * n->n_out, y_dev, n->st);
  MCHK(n, hipGetLastError());
  MCHK(n, hipStreamSynchronize(n->st));
  return DD_OK;
}

// loss and gradient of the masked MSE into n->g
static dd_status loss_grad(dd_mlp* n, const float* x_dev, const float* t_dev,
                           const float* mask_dev, int n_rows, float* loss) {
  const int R = (n_rows + 63) / 64 * 64;
  dd_status s = ensure_rows(n, R);
  if (s) return s;
  mlpk::launch_to_bf16_pad(x_dev, n_rows, n->n_in, R, n->n_in, n->xb, n->st);
  forward_padded(n, R);
  mlpk::launch_mse(n->y, t_dev, mask_dev, n_rows, R, n->n_out, n->gy, n->part, n->scal, n->st);
  // backward: layer l has input act[l] (BF16, R x dims[l]) and output gradient gl (BF16)
  const unsigned short* act[4] = {n->xb, n->hb[0], n->hb[1], n->hb[2]};
  const unsigned short* gl = n->gy;
  for (int l = 3; l >= 0; l--) {
    const int din = n->dims[l], dout = n->dims[l + 1];
    mlpk::Epilogue ew{};
    ew.out_f32 = n->g + n->off_w[l];  // dW = act^T gl  (din x dout)
    mlpk::launch_gemm(true, false, act[l], din, gl, dout, din, dout, R, ew, n->ksplit, n->st);
    mlpk::launch_bias_grad(gl, R, dout, n->g + n->off_b[l], n->st);
    if (l > 0) {
      mlpk::Epilogue eh{};
      eh.out_f32 = n->dh;  // dh = gl W^T  (R x din)
      mlpk::launch_gemm(false, true, gl, dout, n->wb + n->off_w[l], dout, R, din, dout, eh,
                        nullptr, n->st);
      mlpk::launch_relu_back(n->dh, n->z[l - 1], (size_t)R * din, n->dz, n->st);
      gl = n->dz;
    }
  }
  MCHK(n, hipGetLastError());
  MCHK(n, hipMemcpyAsync(n->hscal, n->scal, sizeof(float), hipMemcpyDeviceToHost, n->st));
  MCHK(n, hipStreamSynchronize(n->st));
  if (loss) *loss = n->hscal[0];
  return DD_OK;
}

extern "C" dd_status dd_mlp_loss_grad(dd_mlp* n, const float* x_dev, const float* t_dev,
                                      const float* mask_dev, int n_rows, float* loss,
                                      float* grad_host) {
  if (!n || n_rows <= 0 || !x_dev || !t_dev || !mask_dev) return DD_EINVAL;
  dd_status s = loss_grad(n, x_dev, t_dev, mask_dev, n_rows, loss);
  if (s) return s;
  if (grad_host) {
    MCHK(n, hipMemcpyAsync(grad_host, n->g, sizeof(float) * n->n_params, hipMemcpyDeviceToHost,
                           n->st));
    MCHK(n, hipStreamSynchronize(n->st));
  }
  return DD_OK;
}

extern "C" dd_status dd_mlp_train_step(dd_mlp* n, const float* x_dev, const float* t_dev,
                                       const float* mask_dev, int n_rows, float lr, float* loss) {
  if (!n || n_rows <= 0 || !x_dev || !t_dev || !mask_dev || !(lr > 0)) return DD_EINVAL;
  dd_status s = loss_grad(n, x_dev, t_dev, mask_dev, n_rows, loss);
  if (s) return s;
  n->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f / (1.f - std::pow(b1, (float)n->step));
  const float c2 = 1.f / (1.f - std::pow(b2, (float)n->step));
  mlpk::launch_adam(n->w, n->g, n->m, n->v, n->n_params, lr, b1, b2, 1e-8f, c1, c2, n->wb, n->st);
  MCHK(n, hipGetLastError());
  return DD_OK;
}

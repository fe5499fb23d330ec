// Host runtime of the C-ABI declared in include/dd.h: problem state in HBM,
// the multi-scale schedule driver and the coarse-to-fine refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/dd.h"
#include "../../include/dd_mlp.h"
#include "dd_internal.h"

using ddk::HalfParams;
using ddk::IterStatsDev;
using ddk::kS;

namespace {

thread_local std::string g_init_error;

struct Level {
  int H = 0, W = 0, bh = 0, bw = 0;
  double h = 0;
  double* mu = nullptr;
  double* nu = nullptr;
};

struct Cells {
  int n = 0;
  int4* q = nullptr;
  int2* org = nullptr;
  std::vector<int4> hq;
};

template <typename T>
hipError_t dmalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return hipMalloc((void**)p, sizeof(T) * n);
}

}  // namespace

struct dd_ctx {
  std::string err;
  dd_options opt{};
  hipStream_t st = nullptr;
  int nlev = 0, lev = 0, s = kS;
  double eps = 0;
  std::vector<Level> L;
  std::vector<dd_stage> sched;
  size_t next_stage = 0;
  int last_part = -1;
  // state of the current level
  int nb = 0;
  int64_t* row_off = nullptr;
  int* row_len = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  int64_t capE = 0;
  int64_t nnz = 0;
  double* alpha[2] = {nullptr, nullptr};
  Cells cells[2];
  // sweep scratch
  int cell_cap = 0;
  int64_t* cell_toff = nullptr;
  int* cell_U = nullptr;
  int64_t* cell_ooff = nullptr;
  int* bin_count = nullptr;
  int* bin_list = nullptr;
  double *r_cost = nullptr, *r_obj = nullptr, *r_err = nullptr;
  int *r_loops = nullptr, *r_status = nullptr;
  long long* r_evals = nullptr;
  int* defer_list = nullptr;
  double* defer_F = nullptr;
  long long* misc = nullptr;
  int* uni_key = nullptr;
  double* uni_nu = nullptr;
  double* uni_G = nullptr;
  int64_t capU = 0;
  IterStatsDev* dstats = nullptr;
  IterStatsDev* hstats = nullptr;
  double* dscal = nullptr;
  double* hscal = nullptr;
  double* px_scratch = nullptr;
  int64_t px_cap = 0;
  dd_iter_stats last{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t kev[ddk::kNEvents] = {};
  static_assert(DD_N_KERNELS == ddk::kNKernels, "kernel count of the ABI and the launcher");
  ddk::SweepStreams ss{};
  int* queue = nullptr;
  // warm start by the network
  dd_mlp* warm_net = nullptr;
  int warm_policy = 0;
  float warm_min_rms = 0.f;
  int* warm_count = nullptr;        // cells warm-started, summed over sweeps (device)
  int warm_fresh[2] = {1, 1};     // no sweep of this partition since init/refine/eps change
  unsigned short* warm_X = nullptr;
  float* warm_Y = nullptr;
  int warm_rows = 0;
  double* alpha_prev = nullptr;   // potentials of the partition at the start of the last sweep
  int64_t alpha_prev_cap = 0;
  int* dcount = nullptr;
  hipEvent_t warm_ev[2] = {};
  int n_warm_sweeps = 0;
  int n_cu = 0;
  int stream_wgs = 0;
  float* stream_tile = nullptr;
  float* stream_S = nullptr;
  float* stream_nu = nullptr;
  int grid_cap = 2048;
};

static dd_status fail(dd_ctx* c, dd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c)
    c->err = buf;
  else
    g_init_error = buf;
  return s;
}

#define HIPCHK(c, x)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      return fail((c), e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP, "%s: %s (%s:%d)", \
                  #x, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

// Composite cells as virtual 8x8 pixel blocks: partition A groups basic
// cells {2a, 2a+1} in each direction, partition B {2g-1, 2g} (clipped at the
// border), Sec. 7.1.  Quadrants are stored top-left, top-right, bottom-left,
// bottom-right; absent ones are -1.
static void build_cells(int bh, int bw, int part, std::vector<int4>& q, std::vector<int2>& org) {
  const int gr = part == 0 ? bh / 2 : bh / 2 + 1;
  const int gc = part == 0 ? bw / 2 : bw / 2 + 1;
  q.clear();
  org.clear();
  for (int i = 0; i < gr; i++)
    for (int j = 0; j < gc; j++) {
      const int r0 = part == 0 ? 2 * i : 2 * i - 1;
      const int c0 = part == 0 ? 2 * j : 2 * j - 1;
      int id[4];
      for (int a = 0; a < 4; a++) {
        const int br = r0 + a / 2, bc = c0 + a % 2;
        id[a] = (br >= 0 && br < bh && bc >= 0 && bc < bw) ? br * bw + bc : -1;
      }
      q.push_back(make_int4(id[0], id[1], id[2], id[3]));
      org.push_back(make_int2(r0 * kS, c0 * kS));
    }
}

static dd_status upload_cells(dd_ctx* c) {
  const Level& l = c->L[c->lev];
  for (int p = 0; p < 2; p++) {
    std::vector<int4> q;
    std::vector<int2> org;
    build_cells(l.bh, l.bw, p, q, org);
    Cells& C = c->cells[p];
    hipFree(C.q);
    hipFree(C.org);
    C.q = nullptr;
    C.org = nullptr;
    C.n = (int)q.size();
    HIPCHK(c, dmalloc(&C.q, q.size()));
    HIPCHK(c, dmalloc(&C.org, org.size()));
    HIPCHK(c, hipMemcpyAsync(C.q, q.data(), sizeof(int4) * q.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(C.org, org.data(), sizeof(int2) * org.size(), hipMemcpyHostToDevice,
                             c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    C.hq = q;
  }
  const int need = std::max(c->cells[0].n, c->cells[1].n);
  if (need > c->cell_cap) {
    hipFree(c->cell_toff);
    hipFree(c->cell_U);
    hipFree(c->cell_ooff);
    hipFree(c->bin_list);
    hipFree(c->r_cost);
    hipFree(c->r_obj);
    hipFree(c->r_err);
    hipFree(c->r_loops);
    hipFree(c->r_status);
    hipFree(c->r_evals);
    hipFree(c->defer_list);
    hipFree(c->defer_F);
    HIPCHK(c, dmalloc(&c->cell_toff, need));
    HIPCHK(c, dmalloc(&c->cell_U, need));
    HIPCHK(c, dmalloc(&c->cell_ooff, need));
    HIPCHK(c, dmalloc(&c->bin_list, (size_t)need * ddk::kNBins));
    HIPCHK(c, dmalloc(&c->r_cost, need));
    HIPCHK(c, dmalloc(&c->r_obj, need));
    HIPCHK(c, dmalloc(&c->r_err, need));
    HIPCHK(c, dmalloc(&c->r_loops, need));
    HIPCHK(c, dmalloc(&c->r_status, need));
    HIPCHK(c, dmalloc(&c->r_evals, need));
    HIPCHK(c, dmalloc(&c->defer_list, (size_t)need * ddk::kNDeferGroups));
    HIPCHK(c, dmalloc(&c->defer_F, (size_t)need * 64));
    c->cell_cap = need;
  }
  return DD_OK;
}

// Make the entry buffer hold at least `need` entries, keeping its contents.
static dd_status ensure_entries(dd_ctx* c, int64_t need) {
  if (need <= c->capE) return DD_OK;
  int64_t cap = need + need / 4 + 4096;
  int* col = nullptr;
  double* val = nullptr;
  HIPCHK(c, dmalloc(&col, cap));
  HIPCHK(c, dmalloc(&val, cap));
  if (c->capE > 0) {
    HIPCHK(c, hipMemcpyAsync(col, c->col, sizeof(int) * c->capE, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(val, c->val, sizeof(double) * c->capE, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  hipFree(c->col);
  hipFree(c->val);
  c->col = col;
  c->val = val;
  c->capE = cap;
  return DD_OK;
}

static dd_status ensure_union(dd_ctx* c, int64_t need) {
  if (need <= c->capU) return DD_OK;
  int64_t cap = need + need / 4 + 4096;
  hipFree(c->uni_key);
  hipFree(c->uni_nu);
  hipFree(c->uni_G);
  HIPCHK(c, dmalloc(&c->uni_key, cap));
  HIPCHK(c, dmalloc(&c->uni_nu, cap));
  HIPCHK(c, dmalloc(&c->uni_G, cap));
  c->capU = cap;
  return DD_OK;
}

static dd_status ensure_px(dd_ctx* c, int64_t n) {
  if (n <= c->px_cap) return DD_OK;
  hipFree(c->px_scratch);
  HIPCHK(c, dmalloc(&c->px_scratch, n));
  c->px_cap = n;
  return DD_OK;
}

static void free_state(dd_ctx* c) {
  hipFree(c->row_off);
  hipFree(c->row_len);
  hipFree(c->col);
  hipFree(c->val);
  hipFree(c->alpha[0]);
  hipFree(c->alpha[1]);
  c->row_off = nullptr;
  c->row_len = nullptr;
  c->col = nullptr;
  c->val = nullptr;
  c->alpha[0] = c->alpha[1] = nullptr;
  c->capE = 0;
}

extern "C" void dd_options_default(dd_options* o) {
  if (!o) return;
  o->err_tol = 1e-5;
  o->trunc_threshold = 1e-15;
  o->max_sinkhorn_iter = 50000;
  o->safeguard = 1;
  o->accel = 1;
  o->newton_after = 256;
  o->inputs_on_device = 0;
  o->timing = 0;
  o->stream = nullptr;
}

extern "C" void dd_free(dd_ctx* c) {
  if (!c) return;
  if (c->st) hipStreamSynchronize(c->st);
  free_state(c);
  for (auto& l : c->L) {
    hipFree(l.mu);
    hipFree(l.nu);
  }
  for (int p = 0; p < 2; p++) {
    hipFree(c->cells[p].q);
    hipFree(c->cells[p].org);
  }
  hipFree(c->cell_toff);
  hipFree(c->cell_U);
  hipFree(c->cell_ooff);
  hipFree(c->bin_count);
  hipFree(c->bin_list);
  hipFree(c->r_cost);
  hipFree(c->r_obj);
  hipFree(c->r_err);
  hipFree(c->r_loops);
  hipFree(c->r_status);
  hipFree(c->r_evals);
  hipFree(c->defer_list);
  hipFree(c->defer_F);
  hipFree(c->misc);
  hipFree(c->queue);
  hipFree(c->warm_X);
  hipFree(c->warm_Y);
  hipFree(c->warm_count);
  hipFree(c->alpha_prev);
  hipFree(c->dcount);
  hipFree(c->stream_tile);
  hipFree(c->stream_S);
  hipFree(c->stream_nu);
  hipFree(c->uni_key);
  hipFree(c->uni_nu);
  hipFree(c->uni_G);
  hipFree(c->dstats);
  hipFree(c->dscal);
  hipFree(c->px_scratch);
  if (c->hstats) hipHostFree(c->hstats);
  if (c->hscal) hipHostFree(c->hscal);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  for (int i = 0; i < 3; i++) {
    if (c->ss.aux[i]) hipStreamDestroy(c->ss.aux[i]);
    if (c->ss.join[i]) hipEventDestroy(c->ss.join[i]);
  }
  if (c->ss.fork) hipEventDestroy(c->ss.fork);
  for (auto& e : c->warm_ev)
    if (e) hipEventDestroy(e);
  for (auto& e : c->kev)
    if (e) hipEventDestroy(e);
  delete c;
}

extern "C" const char* dd_last_error(const dd_ctx* c) {
  return c ? c->err.c_str() : g_init_error.c_str();
}

// Product coupling nu_i = |mu_i| nu on level 0 with zero potentials
// (Sec. 6.4: the canonical feasible start without prior knowledge).
static dd_status init_level0(dd_ctx* c) {
  const Level& l = c->L[0];
  const int64_t npx = (int64_t)l.H * l.W;
  std::vector<double> mu(npx), nu(npx);
  HIPCHK(c, hipMemcpyAsync(mu.data(), l.mu, sizeof(double) * npx, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(nu.data(), l.nu, sizeof(double) * npx, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  std::vector<int> ypos;
  for (int64_t p = 0; p < npx; p++)
    if (nu[p] > 0) ypos.push_back((int)p);
  c->nb = l.bh * l.bw;
  std::vector<double> bm(c->nb, 0.0);
  for (int b = 0; b < c->nb; b++) {
    const int br = b / l.bw, bc = b % l.bw;
    double m = 0;
    for (int i = 0; i < kS; i++)
      for (int j = 0; j < kS; j++) m += mu[(int64_t)(br * kS + i) * l.W + bc * kS + j];
    bm[b] = m;
  }
  const int nzy = (int)ypos.size();
  c->nnz = (int64_t)c->nb * nzy;
  HIPCHK(c, dmalloc(&c->row_off, c->nb));
  HIPCHK(c, dmalloc(&c->row_len, c->nb));
  dd_status s = ensure_entries(c, 4 * c->nnz);
  if (s) return s;
  int* dy = nullptr;
  double* dbm = nullptr;
  HIPCHK(c, dmalloc(&dy, nzy));
  HIPCHK(c, dmalloc(&dbm, c->nb));
  HIPCHK(c, hipMemcpyAsync(dy, ypos.data(), sizeof(int) * nzy, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(dbm, bm.data(), sizeof(double) * c->nb, hipMemcpyHostToDevice, c->st));
  ddk::launch_product_init(dy, nzy, l.nu, dbm, c->nb, c->col, c->val, c->row_off, c->row_len,
                           c->st);
  HIPCHK(c, hipGetLastError());
  for (int p = 0; p < 2; p++) {
    HIPCHK(c, dmalloc(&c->alpha[p], npx));
    HIPCHK(c, hipMemsetAsync(c->alpha[p], 0, sizeof(double) * npx, c->st));
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  hipFree(dy);
  hipFree(dbm);
  return upload_cells(c);
}

extern "C" dd_status dd_init(const double* mu, const double* nu, int H, int W, int s, int nlev,
                             const dd_stage* schedule, int n_stages, const dd_options* opt,
                             dd_ctx** out) {
  if (!out) return fail(nullptr, DD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mu || !nu) return fail(nullptr, DD_EINVAL, "mu/nu is NULL");
  if (s != kS) return fail(nullptr, DD_EINVAL, "basic_cell must be %d", kS);
  if (nlev < 1 || nlev > 16) return fail(nullptr, DD_EINVAL, "n_levels out of range");
  if (H <= 0 || W <= 0 || W > 65536) return fail(nullptr, DD_EINVAL, "bad size");
  const int div = (2 * s) << (nlev - 1);
  if (H % div || W % div)
    return fail(nullptr, DD_EINVAL, "height/width must be divisible by %d", div);
  if (!schedule || n_stages < 1) return fail(nullptr, DD_EINVAL, "empty schedule");
  for (int i = 0; i < n_stages; i++) {
    if (!(schedule[i].eps > 0) || schedule[i].level < 0 || schedule[i].level >= nlev ||
        schedule[i].n_half_iters < 0 || (i > 0 && schedule[i].level < schedule[i - 1].level))
      return fail(nullptr, DD_EINVAL, "invalid schedule row %d", i);
  }
  dd_ctx* c = new dd_ctx();
  if (opt)
    c->opt = *opt;
  else
    dd_options_default(&c->opt);
  if (!(c->opt.err_tol > 0) || !(c->opt.trunc_threshold >= 0) || c->opt.max_sinkhorn_iter < 1 ||
      c->opt.newton_after < 0) {
    delete c;
    return fail(nullptr, DD_EINVAL, "invalid options");
  }
  c->st = (hipStream_t)c->opt.stream;
  c->nlev = nlev;
  c->sched.assign(schedule, schedule + n_stages);
  c->eps = schedule[0].eps;
  c->L.resize(nlev);
  const int mx = std::max(H, W);
  auto bail = [&](dd_status st) {
    g_init_error = c->err;
    dd_free(c);
    return st;
  };
  for (int i = nlev - 1; i >= 0; i--) {
    Level& l = c->L[i];
    const int f = nlev - 1 - i;
    l.H = H >> f;
    l.W = W >> f;
    l.bh = l.H / kS;
    l.bw = l.W / kS;
    l.h = (double)(1 << f) / mx;
    const size_t n = (size_t)l.H * l.W;
    if (dmalloc(&l.mu, n) != hipSuccess || dmalloc(&l.nu, n) != hipSuccess)
      return bail(fail(c, DD_ENOMEM, "hipMalloc of level %d failed", i));
    if (i == nlev - 1) {
      hipMemcpyKind k = c->opt.inputs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
      if (hipMemcpyAsync(l.mu, mu, sizeof(double) * n, k, c->st) != hipSuccess ||
          hipMemcpyAsync(l.nu, nu, sizeof(double) * n, k, c->st) != hipSuccess)
        return bail(fail(c, DD_EHIP, "copy of mu/nu failed"));
    } else {
      ddk::launch_pyramid(c->L[i + 1].mu, l.mu, l.H, l.W, c->st);
      ddk::launch_pyramid(c->L[i + 1].nu, l.nu, l.H, l.W, c->st);
    }
  }
  if (dmalloc(&c->dscal, 8) != hipSuccess || hipHostMalloc((void**)&c->hscal, sizeof(double) * 8) != hipSuccess ||
      dmalloc(&c->dstats, 1) != hipSuccess ||
      hipHostMalloc((void**)&c->hstats, sizeof(IterStatsDev)) != hipSuccess ||
      dmalloc(&c->misc, 8) != hipSuccess || dmalloc(&c->bin_count, ddk::kNBins) != hipSuccess ||
      dmalloc(&c->queue, 16) != hipSuccess)
    return bail(fail(c, DD_ENOMEM, "hipMalloc failed"));
  hipEventCreate(&c->ev0);
  hipEventCreate(&c->ev1);
  // auxiliary streams of a sweep (default priority; ordered with the
  // context's stream through events only)
  c->ss.main = c->st;
  if (hipEventCreateWithFlags(&c->ss.fork, hipEventDisableTiming) != hipSuccess)
    return bail(fail(c, DD_EHIP, "event creation failed"));
  for (int i = 0; i < 3; i++)
    if (hipStreamCreateWithFlags(&c->ss.aux[i], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ss.join[i], hipEventDisableTiming) != hipSuccess)
      return bail(fail(c, DD_EHIP, "stream creation failed"));
  if (c->opt.timing)
    for (auto& e : c->kev) hipEventCreate(&e);
  // validation of the finest images
  {
    const Level& l = c->L[nlev - 1];
    ddk::launch_validate(l.mu, l.nu, l.H, l.W, c->dscal, c->st);
    if (hipMemcpyAsync(c->hscal, c->dscal, sizeof(double) * 4, hipMemcpyDeviceToHost, c->st) !=
            hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
      return bail(fail(c, DD_EHIP, "validation failed: %s", hipGetErrorString(hipGetLastError())));
    const double sm = c->hscal[0], sn = c->hscal[1], bad = c->hscal[2], mn = c->hscal[3];
    if (bad > 0) return bail(fail(c, DD_EINVAL, "negative or non-finite mass"));
    if (std::fabs(sm - 1) > 1e-9 || std::fabs(sn - 1) > 1e-9)
      return bail(fail(c, DD_EINVAL, "masses must sum to 1 (got %.17g, %.17g)", sm, sn));
    if (!(mn > 0)) return bail(fail(c, DD_EINVAL, "a basic cell of mu has zero mass"));
  }
  int dev = 0, n_cu = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return bail(fail(c, DD_EHIP, "no HIP device"));
  if (n_cu > 0) c->grid_cap = n_cu * 8;
  c->n_cu = n_cu > 0 ? n_cu : 64;
  {
    const size_t need = ddk::sweep_max_static_lds();
    if (need == 0 || need > (size_t)lds_max)
      return bail(fail(c, DD_EHIP, "kernels need %zu bytes of LDS per workgroup, device allows %d",
                       need, lds_max));
  }
  c->lev = 0;
  dd_status st = init_level0(c);
  if (st) return bail(st);
  *out = c;
  return DD_OK;
}

extern "C" dd_status dd_set_eps(dd_ctx* c, double eps) {
  if (!c) return DD_EINVAL;
  if (!(eps > 0)) return fail(c, DD_EINVAL, "eps must be positive");
  if (eps != c->eps) c->warm_fresh[0] = c->warm_fresh[1] = 1;
  c->eps = eps;
  return DD_OK;
}

static HalfParams make_params(dd_ctx* c, int part) {
  const Level& l = c->L[c->lev];
  HalfParams p{};
  p.H = l.H;
  p.W = l.W;
  p.bh = l.bh;
  p.bw = l.bw;
  p.n_cells = c->cells[part].n;
  p.n_basic = c->nb;
  p.part = part;
  p.h = l.h;
  p.eps = c->eps;
  p.lam = l.h * l.h / c->eps;
  p.err_tol = c->opt.err_tol;
  p.trunc = c->opt.trunc_threshold;
  p.max_iter = c->opt.max_sinkhorn_iter;
  p.safeguard = c->opt.safeguard;
  p.accel = c->opt.accel;
  p.newton_after = c->opt.newton_after;
  p.mu = l.mu;
  p.nu = l.nu;
  p.alpha = c->alpha[part];
  p.cell_q = c->cells[part].q;
  p.cell_org = c->cells[part].org;
  p.row_off = c->row_off;
  p.row_len = c->row_len;
  p.ent_col = c->col;
  p.ent_val = c->val;
  p.cell_toff = c->cell_toff;
  p.cell_U = c->cell_U;
  p.cell_ooff = c->cell_ooff;
  p.bin_count = c->bin_count;
  p.bin_list = c->bin_list;
  p.uni_key = c->uni_key;
  p.uni_nu = c->uni_nu;
  p.uni_G = c->uni_G;
  p.r_cost = c->r_cost;
  p.r_obj = c->r_obj;
  p.r_err = c->r_err;
  p.r_loops = c->r_loops;
  p.r_status = c->r_status;
  p.r_evals = c->r_evals;
  p.misc = c->misc;
  p.queue = c->queue;
  p.stream_tile = c->stream_tile;
  p.stream_S = c->stream_S;
  p.stream_nu = c->stream_nu;
  p.stream_wgs = c->stream_wgs;
  p.defer_list = c->defer_list;
  p.defer_F = c->defer_F;
  p.capE = c->capE;
  return p;
}

// Tile buffers of the streamed solver: one per workgroup (2 MiB each).  The
// workgroups loop over the bin's queue, so fewer of them than cells is still
// correct; size for the bin's cells in the previous sweep plus a margin (64
// before any sweep), at most two per compute unit.
static dd_status ensure_stream(dd_ctx* c, int n_cells) {
  const int prev = c->last.n_cells > 0 ? c->last.cells_bin[ddk::kNBins - 2] + 16 : 64;
  const int want = std::min(std::min(n_cells, 2 * c->n_cu), prev);
  if (want <= c->stream_wgs) return DD_OK;
  hipFree(c->stream_tile);
  hipFree(c->stream_S);
  hipFree(c->stream_nu);
  c->stream_tile = nullptr;
  c->stream_S = nullptr;
  c->stream_nu = nullptr;
  c->stream_wgs = 0;
  HIPCHK(c, dmalloc(&c->stream_tile, (size_t)want * ddk::kStreamTileFloats));
  HIPCHK(c, dmalloc(&c->stream_S, (size_t)want * ddk::kStreamMaxU));
  HIPCHK(c, dmalloc(&c->stream_nu, (size_t)want * ddk::kStreamMaxU));
  c->stream_wgs = want;
  return DD_OK;
}

// Workgroups per solver launch: every workgroup loops over its bin's queue,
// so a launch needs no more workgroups than the GPU holds at once (8 per
// compute unit) or than its bin has cells.  (Sharing the wave slots out in
// proportion to each bin's work in the previous sweep was measured slower.)
static ddk::SweepGrid plan_grid(const dd_ctx* c, int n_cells) {
  ddk::SweepGrid gr{};
  const int g = std::max(1, std::min(n_cells, c->grid_cap));
  for (int b = 0; b < ddk::kNBins; b++) gr.bin[b] = g;
  gr.newton = std::max(1, std::min(n_cells, 2 * c->n_cu));
  gr.other = g;
  return gr;
}

// Warm start of the eligible cells of this sweep: features (BF16 rows), the
// network's forward pass on its own stream (ordered with ours through events),
// and the predicted potential written over alpha.
static dd_status warm_start(dd_ctx* c, const HalfParams& p) {
  const int rows = (p.n_cells + 63) / 64 * 64;
  if (rows > c->warm_rows) {
    hipFree(c->warm_X);
    hipFree(c->warm_Y);
    c->warm_X = nullptr;
    c->warm_Y = nullptr;
    c->warm_rows = 0;
    HIPCHK(c, dmalloc(&c->warm_X, (size_t)rows * ddk::kFeatIn));
    HIPCHK(c, dmalloc(&c->warm_Y, (size_t)rows * 64));
    HIPCHK(c, hipMemsetAsync(c->warm_X, 0, sizeof(unsigned short) * rows * ddk::kFeatIn, c->st));
    c->warm_rows = rows;
  }
  if (!c->warm_ev[0]) {
    HIPCHK(c, hipEventCreateWithFlags(&c->warm_ev[0], hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->warm_ev[1], hipEventDisableTiming));
  }
  ddk::launch_warm_features(p, c->warm_X, c->st);
  hipStream_t ns = (hipStream_t)dd_mlp_get_stream(c->warm_net);
  HIPCHK(c, hipEventRecord(c->warm_ev[0], c->st));
  HIPCHK(c, hipStreamWaitEvent(ns, c->warm_ev[0], 0));
  if (dd_mlp_forward_bf16(c->warm_net, c->warm_X, rows, c->warm_Y) != DD_OK)
    return fail(c, DD_EHIP, "warm-start network: %s", dd_mlp_last_error(c->warm_net));
  HIPCHK(c, hipEventRecord(c->warm_ev[1], ns));
  HIPCHK(c, hipStreamWaitEvent(c->st, c->warm_ev[1], 0));
  if (!c->warm_count) {
    HIPCHK(c, dmalloc(&c->warm_count, 1));
    HIPCHK(c, hipMemsetAsync(c->warm_count, 0, sizeof(int), c->st));
  }
  ddk::launch_warm_apply(p, c->warm_Y, c->warm_min_rms, c->warm_count, c->st);
  HIPCHK(c, hipGetLastError());
  return DD_OK;
}

extern "C" dd_status dd_set_warm_start(dd_ctx* c, dd_mlp* net, int policy, float min_rms) {
  if (!c || policy < 0 || policy > 2 || !(min_rms >= 0)) return DD_EINVAL;
  if (net) {
    int n_in = 0, n_out = 0;
    dd_mlp_shape(net, &n_in, &n_out, nullptr, nullptr);
    if (n_in != ddk::kFeatIn || n_out != 64)
      return fail(c, DD_EINVAL, "warm-start network must map %d features to 64 outputs",
                  ddk::kFeatIn);
  }
  c->warm_net = net;
  c->warm_policy = net ? policy : 0;
  c->warm_min_rms = min_rms;
  c->warm_fresh[0] = c->warm_fresh[1] = 1;
  return DD_OK;
}

extern "C" dd_status dd_warm_start_count(dd_ctx* c, int* n_sweeps, long long* n_cells) {
  if (!c) return DD_EINVAL;
  int n = 0;
  if (c->warm_count) {
    HIPCHK(c, hipMemcpyAsync(&n, c->warm_count, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
  }
  if (n_sweeps) *n_sweeps = c->n_warm_sweeps;
  if (n_cells) *n_cells = n;
  return DD_OK;
}

extern "C" dd_status dd_collect_cells(dd_ctx* c, float* x_dev, float* t_dev, float* mask_dev,
                                      int* cell_dev, int cap, int* n_out) {
  if (!c || !n_out || cap < 0 || (cap > 0 && (!x_dev || !t_dev || !mask_dev))) return DD_EINVAL;
  if (c->last_part < 0) return fail(c, DD_ESTATE, "no half-iteration on this level yet");
  if (!c->dcount) HIPCHK(c, dmalloc(&c->dcount, 1));
  HIPCHK(c, hipMemsetAsync(c->dcount, 0, sizeof(int), c->st));
  HalfParams p = make_params(c, c->last_part);
  ddk::launch_collect(p, c->alpha_prev, x_dev, t_dev, mask_dev, cell_dev, cap, c->dcount, c->st);
  HIPCHK(c, hipGetLastError());
  int n = 0;
  HIPCHK(c, hipMemcpyAsync(&n, c->dcount, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  *n_out = n < cap ? n : cap;
  return DD_OK;
}

extern "C" dd_status dd_half_iterate(dd_ctx* c, int part, dd_iter_stats* out) {
  if (!c) return DD_EINVAL;
  if (part != 0 && part != 1) return fail(c, DD_EINVAL, "partition must be 0 or 1");
  dd_status s = ensure_entries(c, 4 * c->nnz + 64);
  if (s) return s;
  s = ensure_union(c, c->nnz + 64);
  if (s) return s;
  s = ensure_stream(c, c->cells[part].n);
  if (s) return s;
  HalfParams p = make_params(c, part);
  HIPCHK(c, hipMemsetAsync(c->misc, 0, sizeof(long long) * 8, c->st));
  HIPCHK(c, hipMemsetAsync(c->queue, 0, sizeof(int) * 16, c->st));
  HIPCHK(c, hipEventRecord(c->ev0, c->st));
  hipEvent_t* kev = c->opt.timing ? c->kev : nullptr;
  const ddk::SweepGrid gr = plan_grid(c, p.n_cells);
  {
    // keep the starting potentials of this sweep (training samples, dd_collect_cells)
    const Level& l = c->L[c->lev];
    const int64_t npx = (int64_t)l.H * l.W;
    if (npx > c->alpha_prev_cap) {
      hipFree(c->alpha_prev);
      c->alpha_prev = nullptr;
      c->alpha_prev_cap = 0;
      HIPCHK(c, dmalloc(&c->alpha_prev, npx));
      c->alpha_prev_cap = npx;
    }
    HIPCHK(c, hipMemcpyAsync(c->alpha_prev, c->alpha[part], sizeof(double) * npx,
                             hipMemcpyDeviceToDevice, c->st));
  }
  ddk::launch_sweep_prep(p, c->ss, gr, kev);
  const bool warm = c->warm_net && c->warm_policy > 0 &&
                    (c->warm_policy == 2 || c->warm_fresh[part]);
  if (warm) {
    dd_status ws = warm_start(c, p);
    if (ws) return ws;
    c->n_warm_sweeps++;
  }
  c->warm_fresh[part] = 0;
  ddk::launch_sweep_solve(p, c->ss, gr, kev);
  HIPCHK(c, hipGetLastError());
  ddk::launch_stats(p, c->dstats, c->st, kev ? kev + 2 * (DD_N_KERNELS - 1) : nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(c->ev1, c->st));
  HIPCHK(c, hipMemcpyAsync(c->hstats, c->dstats, sizeof(IterStatsDev), hipMemcpyDeviceToHost, c->st));
  long long hmisc[3] = {0, 0, 0};
  HIPCHK(c, hipMemcpyAsync(hmisc, c->misc, sizeof(long long) * 3, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (hmisc[2]) return fail(c, DD_ESTATE, "corrupt basic-cell rows detected");
  if (hmisc[1] > c->capE) return fail(c, DD_ECAPACITY, "output entries exceed capacity");
  float ms = 0;
  hipEventElapsedTime(&ms, c->ev0, c->ev1);
  const IterStatsDev& d = *c->hstats;
  dd_iter_stats r{};
  r.n_cells = d.n_cells;
  r.loops_max = d.loops_max;
  r.loops_total = d.loops_total;
  r.n_failed = d.n_failed;
  r.n_safeguard = d.n_safeguard;
  r.n_newton = d.n_newton;
  r.nnz = d.nnz;
  r.entry_evals = d.evals;
  r.cost = d.cost;
  r.obj = d.obj;
  r.err_x = d.err;
  r.ms = ms;
  for (int k = 0; k < DD_N_BINS; k++) {
    r.cells_bin[k] = d.cells_bin[k];
    r.evals_bin[k] = d.evals_bin[k];
  }
  if (kev)
    for (int k = 0; k < DD_N_KERNELS; k++) {
      float t = 0;
      hipEventElapsedTime(&t, kev[2 * k], kev[2 * k + 1]);
      r.ms_kernel[k] = t;
      if (k == 10)  // the Newton launches on the auxiliary streams
        for (int i = 0; i < ddk::kNDeferGroups - 1; i++) {
          float t2 = 0;
          hipEventElapsedTime(&t2, kev[2 * (ddk::kNKernels + i)], kev[2 * (ddk::kNKernels + i) + 1]);
          r.ms_kernel[k] += t2;
        }
    }
  c->nnz = d.nnz;
  c->last = r;
  c->last_part = part;
  if (out) *out = r;
  return d.n_failed > 0 ? DD_ENOTCONV : DD_OK;
}

// Least-squares gluing potential on the cells of partition A (Sec. 6.3):
// min sum_e (V[b_e] - V[a_e] - w_e)^2 by conjugate gradients, mean zero.
// The sign follows the path-product form of the glued scalings,
// V(J2) - V(J1) ~ log q(J1,J2).
static void glue_solve(int n, const std::vector<int>& ea, const std::vector<int>& eb,
                       const std::vector<double>& w, std::vector<double>& V) {
  std::vector<double> rhs(n, 0.0), r(n), p(n), Ap(n);
  V.assign(n, 0.0);
  const size_t ne = w.size();
  for (size_t e = 0; e < ne; e++) {
    rhs[eb[e]] += w[e];
    rhs[ea[e]] -= w[e];
  }
  r = rhs;
  p = rhs;
  double rr = 0;
  for (int i = 0; i < n; i++) rr += r[i] * r[i];
  const double bb = rr;
  for (int it = 0; it < 20 * n + 100 && rr > 1e-28 * bb && rr > 0; it++) {
    std::fill(Ap.begin(), Ap.end(), 0.0);
    for (size_t e = 0; e < ne; e++) {
      const double d = p[eb[e]] - p[ea[e]];
      Ap[eb[e]] += d;
      Ap[ea[e]] -= d;
    }
    double pAp = 0;
    for (int i = 0; i < n; i++) pAp += p[i] * Ap[i];
    if (!(pAp > 0)) break;
    const double a = rr / pAp;
    double rr2 = 0;
    for (int i = 0; i < n; i++) {
      V[i] += a * p[i];
      r[i] -= a * Ap[i];
      rr2 += r[i] * r[i];
    }
    const double beta = rr2 / rr;
    rr = rr2;
    for (int i = 0; i < n; i++) p[i] = r[i] + beta * p[i];
  }
  double mean = 0;
  for (int i = 0; i < n; i++) mean += V[i];
  mean /= n;
  for (int i = 0; i < n; i++) V[i] -= mean;
}

__global__ void k_glue_apply(const double* aA, const double* V, double eps, int Hc, int Wc,
                             double* out) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)Hc * Wc) return;
  const int r = (int)(i / Wc), cc = (int)(i % Wc);
  const int na_c = Wc / (2 * kS);
  out[i] = aA[i] + eps * V[(r / (2 * kS)) * na_c + cc / (2 * kS)];
}

extern "C" dd_status dd_refine(dd_ctx* c) {
  if (!c) return DD_EINVAL;
  if (c->lev >= c->nlev - 1) return fail(c, DD_ESTATE, "already on the finest level");
  const Level& lc = c->L[c->lev];
  const Level& lf = c->L[c->lev + 1];
  ddk::RefineParams R{};
  R.Hc = lc.H;
  R.Wc = lc.W;
  R.bwc = lc.bw;
  R.Hf = lf.H;
  R.Wf = lf.W;
  R.bwf = lf.bw;
  R.n_basic_f = lf.bh * lf.bw;
  R.eps = c->eps;
  R.mu_c = lc.mu;
  R.nu_c = lc.nu;
  R.mu_f = lf.mu;
  R.nu_f = lf.nu;
  R.alpha_a_c = c->alpha[0];
  R.alpha_b_c = c->alpha[1];
  R.row_off_c = c->row_off;
  R.row_len_c = c->row_len;
  R.col_c = c->col;
  R.val_c = c->val;
  // 1. gluing weights per basic cell, then the least-squares potential on the host
  const int nbc = c->nb;
  double* dq = nullptr;
  HIPCHK(c, dmalloc(&dq, 2 * (size_t)nbc));
  ddk::launch_glue_ratios(R, dq, c->st);
  std::vector<double> q(2 * (size_t)nbc);
  HIPCHK(c, hipMemcpyAsync(q.data(), dq, sizeof(double) * 2 * nbc, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  hipFree(dq);
  const int na = c->cells[0].n;
  std::vector<int> cellA(nbc);
  for (int k = 0; k < na; k++) {
    const int4 t = c->cells[0].hq[k];
    const int ids[4] = {t.x, t.y, t.z, t.w};
    for (int a = 0; a < 4; a++)
      if (ids[a] >= 0) cellA[ids[a]] = k;
  }
  std::vector<int> ea, eb;
  std::vector<double> w;
  for (int k = 0; k < c->cells[1].n; k++) {
    const int4 t = c->cells[1].hq[k];
    int ids[4], n = 0;
    const int all[4] = {t.x, t.y, t.z, t.w};
    for (int a = 0; a < 4; a++)
      if (all[a] >= 0) ids[n++] = all[a];
    for (int a = 0; a < n; a++)
      for (int b = a + 1; b < n; b++) {
        ea.push_back(cellA[ids[a]]);
        eb.push_back(cellA[ids[b]]);
        w.push_back(q[2 * ids[a]] + q[2 * ids[b] + 1]);
      }
  }
  std::vector<double> V;
  glue_solve(na, ea, eb, w, V);
  double *dV = nullptr, *fg = nullptr;
  HIPCHK(c, dmalloc(&dV, na));
  HIPCHK(c, dmalloc(&fg, (size_t)lc.H * lc.W));
  HIPCHK(c, hipMemcpyAsync(dV, V.data(), sizeof(double) * na, hipMemcpyHostToDevice, c->st));
  {
    long long n = (long long)lc.H * lc.W;
    hipLaunchKernelGGL(k_glue_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->st,
                       c->alpha[0], dV, c->eps, lc.H, lc.W, fg);
  }
  // 2. fine potentials
  double *fa = nullptr, *fb = nullptr;
  const size_t nf = (size_t)lf.H * lf.W;
  HIPCHK(c, dmalloc(&fa, nf));
  HIPCHK(c, dmalloc(&fb, nf));
  ddk::launch_interp(fg, lc.H, lc.W, fa, fb, lf.H, lf.W, c->st);
  // 3. fine basic marginals
  const int nbf = R.n_basic_f;
  const int64_t nnzf = 16 * c->nnz;
  int64_t* roff = nullptr;
  int* rlen = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  const int64_t capf = 4 * nnzf + nnzf / 4 + 4096;
  HIPCHK(c, dmalloc(&roff, nbf + 1));
  HIPCHK(c, dmalloc(&rlen, nbf));
  HIPCHK(c, dmalloc(&col, capf));
  HIPCHK(c, dmalloc(&val, capf));
  R.row_off_f = roff;
  R.row_len_f = rlen;
  R.col_f = col;
  R.val_f = val;
  ddk::launch_refine_rows(R, c->st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  hipFree(dV);
  hipFree(fg);
  free_state(c);
  c->row_off = roff;
  c->row_len = rlen;
  c->col = col;
  c->val = val;
  c->capE = capf;
  c->alpha[0] = fa;
  c->alpha[1] = fb;
  c->nnz = nnzf;
  c->lev++;
  c->nb = nbf;
  c->last_part = -1;
  c->warm_fresh[0] = c->warm_fresh[1] = 1;
  return upload_cells(c);
}

extern "C" dd_status dd_run_schedule(dd_ctx* c, dd_run_stats* out) {
  if (!c) return DD_EINVAL;
  dd_run_stats rs{};
  const auto t0 = std::chrono::steady_clock::now();
  dd_status worst = DD_OK;
  for (; c->next_stage < c->sched.size(); c->next_stage++) {
    const dd_stage& sg = c->sched[c->next_stage];
    while (c->lev < sg.level) {
      dd_status s = dd_refine(c);
      if (s < 0) return s;
    }
    if (sg.level != c->lev) return fail(c, DD_ESTATE, "schedule level %d below current %d", sg.level, c->lev);
    dd_set_eps(c, sg.eps);
    for (int k = 0; k < sg.n_half_iters; k++) {
      dd_iter_stats it;
      dd_status s = dd_half_iterate(c, k & 1, &it);
      if (s < 0) return s;
      if (s > 0) worst = s;
      rs.n_half_iters++;
      rs.n_cell_solves += it.n_cells;
      rs.loops_total += it.loops_total;
      rs.entry_evals += it.entry_evals;
      rs.n_failed += it.n_failed;
      rs.n_safeguard += it.n_safeguard;
      rs.n_newton += it.n_newton;
      rs.nnz_max = std::max(rs.nnz_max, it.nnz);
      for (int b = 0; b < DD_N_KERNELS; b++) rs.ms_kernel[b] += it.ms_kernel[b];
      for (int b = 0; b < DD_N_BINS; b++) {
        rs.launches_bin[b] += 1;  // every bin's solver is launched each sweep
        rs.evals_bin[b] += it.evals_bin[b];
      }
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  rs.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = rs;
  return worst;
}

extern "C" dd_status dd_cost(dd_ctx* c, dd_cost_report* r) {
  if (!c || !r) return DD_EINVAL;
  const Level& l = c->L[c->lev];
  dd_status s = ensure_px(c, (int64_t)l.H * l.W + 3 * ddk::kDiagBlocks);
  if (s) return s;
  ddk::launch_diag(c->row_off, c->row_len, c->col, c->val, l.mu, l.nu, l.H, l.W, l.bw, c->nb,
                   c->px_scratch, c->dscal, c->st);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->hscal, c->dscal, sizeof(double) * 3, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  memset(r, 0, sizeof(*r));
  r->err_y = c->hscal[0];
  r->mass_drift = c->hscal[1];
  r->nnz = (int64_t)c->hscal[2];
  r->level = c->lev;
  r->eps = c->eps;
  r->last_partition = c->last_part;
  if (c->last_part >= 0) {
    r->cost = c->last.cost;
    r->obj = c->last.obj;
    r->err_x = c->last.err_x;
  }
  return DD_OK;
}

extern "C" dd_status dd_level_info(const dd_ctx* c, int* level, int* H, int* W, int* n_basic,
                                   int* na, int* nbb, double* eps) {
  if (!c) return DD_EINVAL;
  const Level& l = c->L[c->lev];
  if (level) *level = c->lev;
  if (H) *H = l.H;
  if (W) *W = l.W;
  if (n_basic) *n_basic = c->nb;
  if (na) *na = c->cells[0].n;
  if (nbb) *nbb = c->cells[1].n;
  if (eps) *eps = c->eps;
  return DD_OK;
}

extern "C" dd_status dd_export_plan(dd_ctx* c, dd_plan_view* v) {
  if (!c || !v) return DD_EINVAL;
  const Level& l = c->L[c->lev];
  v->level = c->lev;
  v->H = l.H;
  v->W = l.W;
  v->eps = c->eps;
  v->n_basic = c->nb;
  v->nnz = c->nnz;
  if (!v->row_ptr && !v->col && !v->val && !v->alpha_a && !v->alpha_b) return DD_OK;
  int64_t* rp = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  HIPCHK(c, dmalloc(&rp, c->nb + 1));
  HIPCHK(c, dmalloc(&col, c->nnz));
  HIPCHK(c, dmalloc(&val, c->nnz));
  ddk::launch_export(c->row_off, c->row_len, c->col, c->val, c->nb, rp, col, val, c->st);
  HIPCHK(c, hipGetLastError());
  if (v->row_ptr)
    HIPCHK(c, hipMemcpyAsync(v->row_ptr, rp, sizeof(int64_t) * (c->nb + 1), hipMemcpyDeviceToHost, c->st));
  if (v->col) HIPCHK(c, hipMemcpyAsync(v->col, col, sizeof(int) * c->nnz, hipMemcpyDeviceToHost, c->st));
  if (v->val) HIPCHK(c, hipMemcpyAsync(v->val, val, sizeof(double) * c->nnz, hipMemcpyDeviceToHost, c->st));
  const size_t npx = (size_t)l.H * l.W;
  if (v->alpha_a)
    HIPCHK(c, hipMemcpyAsync(v->alpha_a, c->alpha[0], sizeof(double) * npx, hipMemcpyDeviceToHost, c->st));
  if (v->alpha_b)
    HIPCHK(c, hipMemcpyAsync(v->alpha_b, c->alpha[1], sizeof(double) * npx, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  hipFree(rp);
  hipFree(col);
  hipFree(val);
  return DD_OK;
}

__global__ void k_rows_from_ptr(const int64_t* rp, int n, int64_t* off, int* len) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  off[i] = rp[i];
  len[i] = (int)(rp[i + 1] - rp[i]);
}

extern "C" dd_status dd_import_state(dd_ctx* c, const dd_plan_view* v) {
  if (!c || !v || !v->row_ptr || !v->alpha_a || !v->alpha_b) return DD_EINVAL;
  if (v->level < 0 || v->level >= c->nlev || !(v->eps > 0))
    return fail(c, DD_EINVAL, "bad level/eps");
  const Level& l = c->L[v->level];
  const int nb = l.bh * l.bw;
  if (v->n_basic != nb || v->H != l.H || v->W != l.W)
    return fail(c, DD_EINVAL, "view geometry does not match level %d", v->level);
  const int64_t nnz = v->row_ptr[nb];
  if (nnz > 0 && (!v->col || !v->val)) return fail(c, DD_EINVAL, "col/val missing");
  free_state(c);
  c->lev = v->level;
  c->eps = v->eps;
  c->nb = nb;
  c->nnz = nnz;
  HIPCHK(c, dmalloc(&c->row_off, nb));
  HIPCHK(c, dmalloc(&c->row_len, nb));
  dd_status s = ensure_entries(c, 4 * nnz + 64);
  if (s) return s;
  int64_t* rp = nullptr;
  HIPCHK(c, dmalloc(&rp, nb + 1));
  HIPCHK(c, hipMemcpyAsync(rp, v->row_ptr, sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, c->st));
  if (nnz > 0) {
    HIPCHK(c, hipMemcpyAsync(c->col, v->col, sizeof(int) * nnz, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->val, v->val, sizeof(double) * nnz, hipMemcpyHostToDevice, c->st));
  }
  hipLaunchKernelGGL(k_rows_from_ptr, dim3((nb + 255) / 256), dim3(256), 0, c->st, rp, nb,
                     c->row_off, c->row_len);
  const size_t npx = (size_t)l.H * l.W;
  for (int p = 0; p < 2; p++) {
    HIPCHK(c, dmalloc(&c->alpha[p], npx));
    HIPCHK(c, hipMemcpyAsync(c->alpha[p], p == 0 ? v->alpha_a : v->alpha_b, sizeof(double) * npx,
                             hipMemcpyHostToDevice, c->st));
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  hipFree(rp);
  c->last_part = -1;
  return upload_cells(c);
}

extern "C" dd_status dd_cell_results(dd_ctx* c, double* cost, double* obj, double* err_x,
                                     int* loops, int* status) {
  if (!c) return DD_EINVAL;
  if (c->last_part < 0) return fail(c, DD_ESTATE, "no half-iteration on this level yet");
  const int n = c->cells[c->last_part].n;
  if (cost) HIPCHK(c, hipMemcpyAsync(cost, c->r_cost, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
  if (obj) HIPCHK(c, hipMemcpyAsync(obj, c->r_obj, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
  if (err_x) HIPCHK(c, hipMemcpyAsync(err_x, c->r_err, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
  if (loops) HIPCHK(c, hipMemcpyAsync(loops, c->r_loops, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
  if (status) HIPCHK(c, hipMemcpyAsync(status, c->r_status, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return DD_OK;
}

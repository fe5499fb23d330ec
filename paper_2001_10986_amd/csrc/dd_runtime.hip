// Host runtime of the C-ABI declared in include/dd.h: problem state in HBM,
// the multi-scale schedule driver and the coarse-to-fine refinement.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
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

// Process-wide cache of device blocks: a schedule allocates and frees the
// same buffers level by level, and the next solve repeats the sizes, so
// freed blocks are kept and handed out again (a block of at least the asked
// size and at most twice it, on the same device).  Taking a block back
// synchronises the device first, as hipFree does, so no queued work can
// still reach a block when it is handed out again.  At most kCacheMaxBytes
// per device are kept; a failed allocation releases the device's cache and
// tries once more.
constexpr size_t kCacheMaxBytes = size_t(16) << 30;

struct BlockCache {
  std::mutex mu;
  std::unordered_map<void*, std::pair<size_t, int>> live;  // block -> (bytes, device)
  std::multimap<std::pair<int, size_t>, void*> idle;       // (device, bytes) -> block
  std::unordered_map<int, size_t> idle_bytes;              // per device
};

BlockCache& block_cache() {
  static BlockCache* bc = new BlockCache;  // never destroyed: blocks live until exit
  return *bc;
}

hipError_t cache_malloc(void** p, size_t bytes) {
  *p = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  BlockCache& bc = block_cache();
  {
    std::lock_guard<std::mutex> lk(bc.mu);
    auto it = bc.idle.lower_bound({dev, bytes});
    if (it != bc.idle.end() && it->first.first == dev && it->first.second <= 2 * bytes) {
      const size_t sz = it->first.second;
      *p = it->second;
      bc.idle.erase(it);
      bc.idle_bytes[dev] -= sz;
      bc.live[*p] = {sz, dev};
      return hipSuccess;
    }
  }
  e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    std::vector<void*> rel;
    {
      std::lock_guard<std::mutex> lk(bc.mu);
      for (auto it = bc.idle.begin(); it != bc.idle.end();) {
        if (it->first.first == dev) {
          rel.push_back(it->second);
          it = bc.idle.erase(it);
        } else {
          ++it;
        }
      }
      bc.idle_bytes[dev] = 0;
    }
    for (void* q : rel) (void)hipFree(q);
    e = hipMalloc(p, bytes);
  }
  if (e != hipSuccess) {
    *p = nullptr;
    return e;
  }
  std::lock_guard<std::mutex> lk(bc.mu);
  bc.live[*p] = {bytes, dev};
  return hipSuccess;
}

// Release a block of cache_malloc (or any device pointer, which goes to hipFree).
void dfree(void* p) {
  if (!p) return;
  BlockCache& bc = block_cache();
  size_t sz = 0;
  int bdev = -1;
  {
    std::lock_guard<std::mutex> lk(bc.mu);
    auto it = bc.live.find(p);
    if (it != bc.live.end()) {
      sz = it->second.first;
      bdev = it->second.second;
      bc.live.erase(it);
    }
  }
  int dev = -1;
  if (bdev < 0 || hipGetDevice(&dev) != hipSuccess || dev != bdev ||
      hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(p);
    return;
  }
  std::lock_guard<std::mutex> lk(bc.mu);
  if (bc.idle_bytes[dev] + sz > kCacheMaxBytes) {
    (void)hipFree(p);  // synchronised above, so nothing queued reaches it
    return;
  }
  bc.idle.insert({{dev, sz}, p});
  bc.idle_bytes[dev] += sz;
}

template <typename T>
hipError_t dmalloc(T** p, size_t n) {
  *p = nullptr;
  if (n == 0) n = 1;
  return cache_malloc((void**)p, sizeof(T) * n);
}

// Work lists, streams and events through which the sweeps of one or more
// problems run: a context runs its own sweeps through one, a batch of
// contexts through another.
struct Runner {
  hipStream_t main = nullptr;
  ddk::SweepStreams ss{};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t kev[ddk::kNEvents] = {};
  bool timing = false;
  int n_cu = 64;
  int solver_per_cu = 8;           // workgroups per solver launch, per compute unit
  int newton_per_cu = 2;           // workgroups per Newton launch, per compute unit
  int stream_max = 0;              // workgroups of the streamed solver at most (0: 2 per CU)
  int wg_cells = 0;                // register solvers: cells per workgroup (0: persistent)
  int n_cap = 0;                   // problems the parameter and statistics arrays hold
  HalfParams* dP = nullptr;        // per-problem parameters (device)
  HalfParams* hP = nullptr;        // their pinned host staging
  IterStatsDev* dstats = nullptr;  // per-problem statistics of the last sweep (device)
  IterStatsDev* hstats = nullptr;  // pinned host copy
  int cap = 0;                     // items each work list holds
  int* bin_count = nullptr;
  int* bin_list = nullptr;
  int* queue = nullptr;
  int* defer_count = nullptr;
  int* defer_list = nullptr;
  int stream_wgs = 0;
  int stream_prev = -1;            // streamed-solver cells of the last sweep (-1: none yet)
  int big_prev = -1;               // log-domain-bin cells of the last sweep (-1: unknown)
  float* stream_tile = nullptr;
  float* stream_S = nullptr;
  float* stream_nu = nullptr;
};

static void runner_free(Runner& r) {
  if (r.main) (void)hipStreamSynchronize(r.main);
  for (int i = 0; i < 3; i++) {
    if (r.ss.aux[i]) (void)hipStreamSynchronize(r.ss.aux[i]);
    if (r.ss.aux[i]) (void)hipStreamDestroy(r.ss.aux[i]);
    if (r.ss.join[i]) (void)hipEventDestroy(r.ss.join[i]);
  }
  if (r.ss.fork) (void)hipEventDestroy(r.ss.fork);
  if (r.ev0) (void)hipEventDestroy(r.ev0);
  if (r.ev1) (void)hipEventDestroy(r.ev1);
  for (auto& e : r.kev)
    if (e) (void)hipEventDestroy(e);
  (void)dfree(r.dP);
  (void)dfree(r.dstats);
  if (r.hP) (void)hipHostFree(r.hP);
  if (r.hstats) (void)hipHostFree(r.hstats);
  (void)dfree(r.bin_count);
  (void)dfree(r.bin_list);
  (void)dfree(r.queue);
  (void)dfree(r.defer_count);
  (void)dfree(r.defer_list);
  (void)dfree(r.stream_tile);
  (void)dfree(r.stream_S);
  (void)dfree(r.stream_nu);
  r = Runner();
}

// Streams (default priority; ordered with `main` through events only),
// events and the fixed-size counters.
static hipError_t runner_init(Runner& r, hipStream_t main, bool timing) {
  r.main = main;
  r.ss.main = main;
  r.timing = timing;
  hipError_t e;
  if ((e = hipEventCreateWithFlags(&r.ss.fork, hipEventDisableTiming)) != hipSuccess) return e;
  for (int i = 0; i < 3; i++) {
    if ((e = hipStreamCreateWithFlags(&r.ss.aux[i], hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&r.ss.join[i], hipEventDisableTiming)) != hipSuccess) return e;
  }
  if ((e = hipEventCreate(&r.ev0)) != hipSuccess || (e = hipEventCreate(&r.ev1)) != hipSuccess)
    return e;
  if (timing)
    for (auto& ev : r.kev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) return e;
  int dev = 0, n_cu = 0;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
    return e;
  if (n_cu > 0) r.n_cu = n_cu;
  if ((e = dmalloc(&r.bin_count, ddk::kNBins)) != hipSuccess) return e;
  if ((e = dmalloc(&r.queue, ddk::kNBins + ddk::kNDeferGroups)) != hipSuccess) return e;
  return dmalloc(&r.defer_count, ddk::kNDeferGroups);
}

// Room for n_prob problems and `items` cells per sweep.
static hipError_t runner_reserve(Runner& r, int n_prob, int items) {
  hipError_t e;
  if (n_prob > r.n_cap) {
    dfree(r.dP);
    dfree(r.dstats);
    if (r.hP) hipHostFree(r.hP);
    if (r.hstats) hipHostFree(r.hstats);
    r.dP = nullptr;
    r.dstats = nullptr;
    r.hP = nullptr;
    r.hstats = nullptr;
    r.n_cap = 0;
    if ((e = dmalloc(&r.dP, n_prob)) != hipSuccess) return e;
    if ((e = dmalloc(&r.dstats, n_prob)) != hipSuccess) return e;
    if ((e = hipHostMalloc((void**)&r.hP, sizeof(HalfParams) * n_prob)) != hipSuccess) return e;
    if ((e = hipHostMalloc((void**)&r.hstats, sizeof(IterStatsDev) * n_prob)) != hipSuccess)
      return e;
    r.n_cap = n_prob;
  }
  if (items > r.cap) {
    dfree(r.bin_list);
    dfree(r.defer_list);
    r.bin_list = nullptr;
    r.defer_list = nullptr;
    r.cap = 0;
    if ((e = dmalloc(&r.bin_list, (size_t)items * ddk::kNBins)) != hipSuccess) return e;
    if ((e = dmalloc(&r.defer_list, (size_t)items * ddk::kNDeferGroups)) != hipSuccess) return e;
    r.cap = items;
  }
  return hipSuccess;
}

// Tile buffers of the streamed solver: one per workgroup (2 MiB each).  The
// workgroups loop over the bin's queue, so fewer of them than cells is still
// correct; size for the bin's cells in the previous sweep plus a margin (64
// before any sweep), at most two per compute unit.  The tuned cap keeps a
// large bin's tiles from competing for the caches; a bin that held at most
// kStreamOwnWg cells in the previous sweep (the coarse levels, where the
// partitions alternate between, e.g., 64 and 81 such cells) gets up to
// kStreamOwnWg workgroups, one per cell, instead of a second round.
constexpr int kStreamOwnWg = 128;

static bool stream_small(const Runner& r) {
  return r.stream_prev >= 0 && r.stream_prev <= kStreamOwnWg;
}

static int stream_limit(const Runner& r) {
  const int tuned = r.stream_max > 0 ? r.stream_max : 2 * r.n_cu;
  return stream_small(r) ? std::max(tuned, kStreamOwnWg) : tuned;
}

static hipError_t runner_stream(Runner& r, int n_cells) {
  const int prev = stream_small(r) ? kStreamOwnWg : r.stream_prev >= 0 ? r.stream_prev + 16 : 64;
  const int want = std::min(std::min(n_cells, stream_limit(r)), prev);
  if (want <= r.stream_wgs) return hipSuccess;
  dfree(r.stream_tile);
  dfree(r.stream_S);
  dfree(r.stream_nu);
  r.stream_tile = nullptr;
  r.stream_S = nullptr;
  r.stream_nu = nullptr;
  r.stream_wgs = 0;
  hipError_t e;
  if ((e = dmalloc(&r.stream_tile, (size_t)want * ddk::kStreamTileFloats)) != hipSuccess) return e;
  if ((e = dmalloc(&r.stream_S, (size_t)want * ddk::kStreamMaxU)) != hipSuccess) return e;
  if ((e = dmalloc(&r.stream_nu, (size_t)want * ddk::kStreamMaxU)) != hipSuccess) return e;
  r.stream_wgs = want;
  return hipSuccess;
}

static ddk::SweepSched runner_sched(const Runner& r, int n_prob, bool quad) {
  ddk::SweepSched sc{};
  sc.n_prob = n_prob;
  sc.quad = quad ? 1 : 0;
  sc.cap = r.cap;
  sc.bin_count = r.bin_count;
  sc.bin_list = r.bin_list;
  sc.queue = r.queue;
  sc.defer_count = r.defer_count;
  sc.defer_list = r.defer_list;
  sc.stream_tile = r.stream_tile;
  sc.stream_S = r.stream_S;
  sc.stream_nu = r.stream_nu;
  sc.stream_wgs = r.stream_wgs;
  sc.wg_cells = r.wg_cells;
  return sc;
}

// Workgroups per solver launch: every workgroup loops over its bin's queue,
// so a launch needs no more workgroups than the GPU holds at once or than its
// bin has cells; the counts per compute unit are set by dd_set_launch or
// picked by dd_autotune (default 8 per solver launch, 2 per Newton launch).
// The union kernel runs a row of workgroups per problem.
static ddk::SweepGrid plan_grid(const Runner& r, int total_cells, int max_cells, int n_prob) {
  ddk::SweepGrid gr{};
  const int cap = r.solver_per_cu * r.n_cu;
  const int g = std::max(1, std::min(total_cells, cap));
  for (int b = 0; b < ddk::kNBins; b++) gr.bin[b] = g;
  // one-shot register-solver workgroups: enough of them for every cell
  if (r.wg_cells > 0)
    for (int b = 0; b < ddk::kNRegBins; b++)
      gr.bin[b] = std::max(1, (total_cells + r.wg_cells - 1) / r.wg_cells);
  // the streamed solver's tiles (up to 2 MiB each) are re-read every loop:
  // fewer workgroups keep more of them in the last-level cache
  gr.bin[ddk::kNBins - 2] = std::min(g, stream_limit(r));
  // the log-domain bin is usually empty, and an empty persistent grid still
  // waits for compute units behind the other bins' workgroups: size it from
  // the last sweep's count (kept unknown across refinements and growing eps)
  if (r.big_prev >= 0) gr.bin[ddk::kNBins - 1] = std::min(g, std::max(32, r.big_prev + 16));
  gr.newton = std::max(1, std::min(total_cells, r.newton_per_cu * r.n_cu));
  gr.other = std::max(1, std::min(max_cells, std::max(64, 8 * r.n_cu / std::max(n_prob, 1))));
  return gr;
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
  double* defer_F = nullptr;
  long long* misc = nullptr;
  int* uni_key = nullptr;
  double* uni_nu = nullptr;
  double* uni_G = nullptr;
  int64_t capU = 0;
  double* dscal = nullptr;
  double* hscal = nullptr;
  double* px_scratch = nullptr;
  int64_t px_cap = 0;
  dd_iter_stats last{};
  double last_eps = 0;  // eps of the half-iteration whose results `last` holds
  int device = 0;                  // HIP device the context was created on
  double* noalloc_scratch = nullptr;  // device address of this device's dd_cost_noalloc scratch
  int refine_glue_iters = 0;       // CG steps of the last refinement's gluing solve
  double refine_glue_resid = 0;    // and its final relative residual
  static_assert(DD_N_KERNELS == ddk::kNKernels, "kernel count of the ABI and the launcher");
  Runner run;  // this context's own sweeps
  // warm start by the network
  dd_mlp* warm_net = nullptr;
  int warm_policy = 0;
  float warm_min_rms = 0.f;
  int* warm_count = nullptr;        // cells warm-started, summed over sweeps (device)
  const float* warm_given = nullptr;  // one-shot prediction for the next sweep (caller's device rows)
  float warm_given_rms = 0.f;
  int warm_fresh[2] = {1, 1};     // no sweep of this partition since init/refine/eps change
  int warm_level[2] = {1, 1};     // no sweep of this partition since init/refine
  unsigned short* warm_X = nullptr;
  float* warm_Y = nullptr;
  int warm_rows = 0;
  double* alpha_prev = nullptr;   // potentials of the partition at the start of the last sweep
  int64_t alpha_prev_cap = 0;
  int* dcount = nullptr;
  hipEvent_t warm_ev[2] = {};
  int n_warm_sweeps = 0;
  bool in_batch = false;  // sweeps run through a batch (dd_batch_create .. dd_batch_free)
  bool prev_valid = false;  // alpha_prev holds the starting potentials of the last sweep
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
static void build_cells(int bh, int bw, int part, int s, std::vector<int4>& q,
                        std::vector<int2>& org) {
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
      org.push_back(make_int2(r0 * s, c0 * s));
    }
}

static dd_status upload_cells(dd_ctx* c) {
  const Level& l = c->L[c->lev];
  for (int p = 0; p < 2; p++) {
    std::vector<int4> q;
    std::vector<int2> org;
    build_cells(l.bh, l.bw, p, c->s, q, org);
    Cells& C = c->cells[p];
    dfree(C.q);
    dfree(C.org);
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
    dfree(c->cell_toff);
    dfree(c->cell_U);
    dfree(c->cell_ooff);
    dfree(c->bin_list);
    dfree(c->r_cost);
    dfree(c->r_obj);
    dfree(c->r_err);
    dfree(c->r_loops);
    dfree(c->r_status);
    dfree(c->r_evals);
    dfree(c->defer_F);
    HIPCHK(c, dmalloc(&c->cell_toff, need));
    HIPCHK(c, dmalloc(&c->cell_U, need));
    HIPCHK(c, dmalloc(&c->cell_ooff, need));
    HIPCHK(c, dmalloc(&c->bin_list, (size_t)need * ddk::kNBins));
    HIPCHK(c, dmalloc(&c->r_cost, need));
    HIPCHK(c, dmalloc(&c->r_obj, need));
    HIPCHK(c, dmalloc(&c->r_err, need));
    HIPCHK(c, dmalloc(&c->r_loops, need));
    HIPCHK(c, dmalloc(&c->r_status, need));
    HIPCHK(c, dmalloc(&c->r_evals, 3 * (size_t)need));  // + Newton-launch work (2 arrays)
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
  dfree(c->col);
  dfree(c->val);
  c->col = col;
  c->val = val;
  c->capE = cap;
  return DD_OK;
}

static dd_status ensure_union(dd_ctx* c, int64_t need) {
  if (need <= c->capU) return DD_OK;
  int64_t cap = need + need / 4 + 4096;
  dfree(c->uni_key);
  dfree(c->uni_nu);
  dfree(c->uni_G);
  HIPCHK(c, dmalloc(&c->uni_key, cap));
  HIPCHK(c, dmalloc(&c->uni_nu, cap));
  HIPCHK(c, dmalloc(&c->uni_G, cap));
  c->capU = cap;
  return DD_OK;
}

static dd_status ensure_px(dd_ctx* c, int64_t n) {
  if (n <= c->px_cap) return DD_OK;
  dfree(c->px_scratch);
  HIPCHK(c, dmalloc(&c->px_scratch, n));
  c->px_cap = n;
  return DD_OK;
}

static void free_state(dd_ctx* c) {
  dfree(c->row_off);
  dfree(c->row_len);
  dfree(c->col);
  dfree(c->val);
  dfree(c->alpha[0]);
  dfree(c->alpha[1]);
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
  o->newton_after = 384;
  o->precision = DD_PREC_SPLIT;
  o->inputs_on_device = 0;
  o->timing = 0;
  o->stream = nullptr;
  o->cost_p = 2.0;
  o->safeguard_after = 1024;
}

extern "C" void dd_free(dd_ctx* c) {
  if (!c) return;
  if (c->st) hipStreamSynchronize(c->st);
  free_state(c);
  for (auto& l : c->L) {
    dfree(l.mu);
    dfree(l.nu);
  }
  for (int p = 0; p < 2; p++) {
    dfree(c->cells[p].q);
    dfree(c->cells[p].org);
  }
  dfree(c->cell_toff);
  dfree(c->cell_U);
  dfree(c->cell_ooff);
  dfree(c->bin_count);
  dfree(c->bin_list);
  dfree(c->r_cost);
  dfree(c->r_obj);
  dfree(c->r_err);
  dfree(c->r_loops);
  dfree(c->r_status);
  dfree(c->r_evals);
  dfree(c->defer_F);
  dfree(c->misc);
  dfree(c->warm_X);
  dfree(c->warm_Y);
  dfree(c->warm_count);
  dfree(c->alpha_prev);
  dfree(c->dcount);
  dfree(c->uni_key);
  dfree(c->uni_nu);
  dfree(c->uni_G);
  dfree(c->dscal);
  dfree(c->px_scratch);
  if (c->hscal) hipHostFree(c->hscal);
  runner_free(c->run);
  for (auto& e : c->warm_ev)
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
    for (int i = 0; i < c->s; i++)
      for (int j = 0; j < c->s; j++) m += mu[(int64_t)(br * c->s + i) * l.W + bc * c->s + j];
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
  dfree(dy);
  dfree(dbm);
  return upload_cells(c);
}

// ---- scratch of the allocation-free diagnostics (dd_cost_noalloc) -------
// The per-pixel Y-marginal accumulator and the block partial sums of the
// diagnostics kernels live in a file-scope device array: one copy on every
// GPU the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol); it uses the device address looked up once per device, with
// that device current, at the first dd_init on it.
constexpr int64_t kNoAllocMaxPx = int64_t(1) << 22;  // 2048 x 2048 pixels
static __device__ __align__(256) double dd_cost_scratch[kNoAllocMaxPx + 3 * ddk::kDiagBlocks];
constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static double* g_noalloc_ptr[kMaxDevices] = {};

static hipError_t noalloc_scratch_ptr(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_noalloc_ptr[dev]) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(dd_cost_scratch));
    if (prev != dev) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}

extern "C" dd_status dd_init(const double* mu, const double* nu, int H, int W, int s, int nlev,
                             const dd_stage* schedule, int n_stages, const dd_options* opt,
                             dd_ctx** out) {
  if (!out) return fail(nullptr, DD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!mu || !nu) return fail(nullptr, DD_EINVAL, "mu/nu is NULL");
  if (s != 2 && s != 4) return fail(nullptr, DD_EINVAL, "basic_cell must be 2 or 4 (got %d)", s);
  if (nlev < 1 || nlev > 16) return fail(nullptr, DD_EINVAL, "n_levels out of range");
  if (opt && !(opt->cost_p > 1.0 && opt->cost_p <= 16.0))
    return fail(nullptr, DD_EINVAL, "cost exponent p must lie in (1, 16] (got %g)", opt->cost_p);
  if (opt && opt->safeguard_after < 0)
    return fail(nullptr, DD_EINVAL, "safeguard_after must be >= 0 (got %d)", opt->safeguard_after);
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
      c->opt.newton_after < 0 ||
      (c->opt.precision != DD_PREC_SPLIT && c->opt.precision != DD_PREC_FP64)) {
    delete c;
    return fail(nullptr, DD_EINVAL, "invalid options");
  }
  c->st = (hipStream_t)c->opt.stream;
  c->nlev = nlev;
  c->s = s;
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
    l.bh = l.H / s;
    l.bw = l.W / s;
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
      dmalloc(&c->misc, 8) != hipSuccess || dmalloc(&c->bin_count, ddk::kNBins) != hipSuccess)
    return bail(fail(c, DD_ENOMEM, "hipMalloc failed"));
  {
    const hipError_t e = runner_init(c->run, c->st, c->opt.timing != 0);
    if (e != hipSuccess)
      return bail(fail(c, DD_EHIP, "stream/event setup failed: %s", hipGetErrorString(e)));
  }
  // validation of the finest images
  {
    const Level& l = c->L[nlev - 1];
    ddk::launch_validate(l.mu, l.nu, c->s, l.H, l.W, c->dscal, c->st);
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
  int dev = 0, lds_max = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return bail(fail(c, DD_EHIP, "no HIP device"));
  c->device = dev;
  {
    const hipError_t e = noalloc_scratch_ptr(dev, &c->noalloc_scratch);
    if (e != hipSuccess)
      return bail(fail(c, DD_EHIP, "address of the static diagnostics scratch: %s",
                       hipGetErrorString(e)));
  }
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
  if (eps > c->eps) c->run.big_prev = -1;  // supports may grow past the last sweep's bins
  c->eps = eps;
  return DD_OK;
}

static HalfParams make_params(dd_ctx* c, int part) {
  const Level& l = c->L[c->lev];
  HalfParams p{};
  p.H = l.H;
  p.s = c->s;
  p.W = l.W;
  p.bh = l.bh;
  p.bw = l.bw;
  p.n_cells = c->cells[part].n;
  p.n_basic = c->nb;
  p.part = part;
  p.h = l.h;
  p.half_p = 0.5 * c->opt.cost_p;
  p.hp = c->opt.cost_p == 2.0 ? l.h * l.h : std::pow(l.h, c->opt.cost_p);
  p.eps = c->eps;
  p.lam = p.hp / c->eps;
  p.err_tol = c->opt.err_tol;
  p.trunc = c->opt.trunc_threshold;
  p.max_iter = c->opt.max_sinkhorn_iter;
  p.safeguard = c->opt.safeguard;
  p.cap0 = p.max_iter;
  if (p.safeguard && c->opt.safeguard_after > 0 && c->opt.safeguard_after < p.cap0)
    p.cap0 = c->opt.safeguard_after;
  p.accel = c->opt.accel;
  p.newton_after = c->opt.newton_after;
  p.fp64 = c->opt.precision == DD_PREC_FP64;
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
  p.r_nev = c->r_evals + c->cell_cap;
  p.r_nmf = c->r_evals + 2 * (size_t)c->cell_cap;
  p.misc = c->misc;
  p.defer_F = c->defer_F;
  p.capE = c->capE;
  return p;
}

// Warm start of the eligible cells of this sweep: features (BF16 rows), the
// network's forward pass on its own stream (ordered with ours through events),
// and the predicted potential written over alpha.
static dd_status warm_start(dd_ctx* c, const HalfParams& p) {
  const int rows = (p.n_cells + 63) / 64 * 64;
  if (rows > c->warm_rows) {
    dfree(c->warm_X);
    dfree(c->warm_Y);
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

extern "C" dd_status dd_set_warm_prediction(dd_ctx* c, const float* y_dev, float min_rms) {
  if (!c || !(min_rms >= 0)) return DD_EINVAL;
  if (c->in_batch) return fail(c, DD_ESTATE, "the context belongs to a batch");
  if (c->s != 4) return fail(c, DD_EINVAL, "predicted starts assume 4x4 basic cells");
  c->warm_given = y_dev;
  c->warm_given_rms = min_rms;
  return DD_OK;
}

extern "C" dd_status dd_set_warm_start(dd_ctx* c, dd_mlp* net, int policy, float min_rms) {
  if (!c || policy < 0 || policy > 3 || !(min_rms >= 0)) return DD_EINVAL;
  if (net && c->opt.cost_p != 2.0)
    return fail(c, DD_EINVAL, "the warm-start network's features assume the quadratic cost");
  if (net && c->s != 4)
    return fail(c, DD_EINVAL, "the warm-start network's features assume 4x4 basic cells");
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
  c->warm_level[0] = c->warm_level[1] = 1;
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
  if (c->s != 4) return fail(c, DD_EINVAL, "cell features assume 4x4 basic cells");
  if (!c->prev_valid)
    return fail(c, DD_ESTATE, "the last sweep ran in a batch; its starting potentials are not kept");
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

// Host side of a sweep of one problem, before its kernels: buffer capacities
// (the output of a sweep needs at most 4 entries per entry it reads), the
// starting potentials kept for dd_collect_cells (keep_prev), and the kernel
// parameters.
static dd_status sweep_begin(dd_ctx* c, int part, bool keep_prev, HalfParams* p) {
  dd_status s = ensure_entries(c, 4 * c->nnz + 64);
  if (s) return s;
  s = ensure_union(c, c->nnz + 64);
  if (s) return s;
  *p = make_params(c, part);
  if (p->n_cells > ddk::kItemCellMask + 1)
    return fail(c, DD_ECAPACITY, "%d cells exceed the %d one sweep can address", p->n_cells,
                ddk::kItemCellMask + 1);
  c->prev_valid = keep_prev;
  if (!keep_prev) return DD_OK;
  const Level& l = c->L[c->lev];
  const int64_t npx = (int64_t)l.H * l.W;
  if (npx > c->alpha_prev_cap) {
    dfree(c->alpha_prev);
    c->alpha_prev = nullptr;
    c->alpha_prev_cap = 0;
    HIPCHK(c, dmalloc(&c->alpha_prev, npx));
    c->alpha_prev_cap = npx;
  }
  HIPCHK(c, hipMemcpyAsync(c->alpha_prev, c->alpha[part], sizeof(double) * npx,
                           hipMemcpyDeviceToDevice, c->st));
  return DD_OK;
}

// Per-kernel times of the last sweep of a runner (timing mode): durations
// and start/end after the sweep's start event; ms_kernel[3 * DD_N_KERNELS].
static void runner_kernel_ms(const Runner& r, double* mk) {
  double* dur = mk;
  double* t0 = mk + DD_N_KERNELS;
  double* t1 = mk + 2 * DD_N_KERNELS;
  auto span = [&](int slot, double* d, double* a, double* b) {
    float s = 0, e = 0;
    (void)hipEventElapsedTime(&s, r.ev0, r.kev[2 * slot]);
    (void)hipEventElapsedTime(&e, r.ev0, r.kev[2 * slot + 1]);
    float t = 0;
    (void)hipEventElapsedTime(&t, r.kev[2 * slot], r.kev[2 * slot + 1]);
    *d += t;
    *a = std::min(*a, (double)s);
    *b = std::max(*b, (double)e);
  };
  for (int k = 0; k < DD_N_KERNELS; k++) {
    dur[k] = 0;
    t0[k] = INFINITY;
    t1[k] = -INFINITY;
    span(k, &dur[k], &t0[k], &t1[k]);
    if (k == 10)  // the Newton launches on the auxiliary streams
      for (int i = 0; i < ddk::kNDeferGroups - 1; i++)
        span(ddk::kNKernels + i, &dur[k], &t0[k], &t1[k]);
  }
}

// Host side of a sweep of one problem, after its statistics came back.
static dd_status sweep_finish(dd_ctx* c, int part, const IterStatsDev& d, float ms,
                              const double* ms_kernel, dd_iter_stats* out) {
  if (d.bad_rows) return fail(c, DD_ESTATE, "corrupt basic-cell rows detected");
  if (d.out_entries > c->capE) return fail(c, DD_ECAPACITY, "output entries exceed capacity");
  dd_iter_stats r{};
  r.n_cells = d.n_cells;
  r.loops_max = d.loops_max;
  r.loops_total = d.loops_total;
  r.n_failed = d.n_failed;
  r.n_safeguard = d.n_safeguard;
  r.n_newton = d.n_newton;
  r.nnz = d.nnz;
  r.entry_evals = d.evals;
  r.newton_evals = d.newton_evals;
  r.newton_mfma_flops = d.newton_mfma;
  r.cost = d.cost;
  r.obj = d.obj;
  r.err_x = d.err;
  r.ms = ms;
  for (int k = 0; k < DD_N_BINS; k++) {
    r.cells_bin[k] = d.cells_bin[k];
    r.evals_bin[k] = d.evals_bin[k];
  }
  if (ms_kernel)
    for (int k = 0; k < DD_N_KERNELS; k++) {
      r.ms_kernel[k] = ms_kernel[k];
      r.ms_start[k] = ms_kernel[DD_N_KERNELS + k];
      r.ms_end[k] = ms_kernel[2 * DD_N_KERNELS + k];
    }
  c->nnz = d.nnz;
  c->last = r;
  c->last_eps = c->eps;
  c->last_part = part;
  if (out) *out = r;
  return d.n_failed > 0 ? DD_ENOTCONV : DD_OK;
}

extern "C" dd_status dd_half_iterate(dd_ctx* c, int part, dd_iter_stats* out) {
  if (!c) return DD_EINVAL;
  if (part != 0 && part != 1) return fail(c, DD_EINVAL, "partition must be 0 or 1");
  if (c->in_batch) return fail(c, DD_ESTATE, "the context belongs to a batch");
  HalfParams p;
  dd_status s = sweep_begin(c, part, true, &p);
  if (s) return s;
  Runner& r = c->run;
  HIPCHK(c, runner_reserve(r, 1, p.n_cells));
  HIPCHK(c, runner_stream(r, p.n_cells));
  r.hP[0] = p;
  HIPCHK(c, hipMemcpyAsync(r.dP, r.hP, sizeof(HalfParams), hipMemcpyHostToDevice, c->st));
  const ddk::SweepSched sc = runner_sched(r, 1, c->opt.cost_p == 2.0);
  const ddk::SweepGrid gr = plan_grid(r, p.n_cells, p.n_cells, 1);
  hipEvent_t* kev = r.timing ? r.kev : nullptr;
  HIPCHK(c, hipEventRecord(r.ev0, c->st));
  ddk::launch_sweep_prep(r.dP, sc, r.ss, gr, kev);
  const bool warm = c->warm_net && c->warm_policy > 0 &&
                    (c->warm_policy == 2 || (c->warm_policy == 1 && c->warm_fresh[part]) ||
                     (c->warm_policy == 3 && c->warm_level[part]));
  if (c->warm_given) {
    // a prediction handed in by dd_set_warm_prediction replaces the network
    // on this sweep (same apply kernel, same eligibility rule)
    if (!c->warm_count) {
      HIPCHK(c, dmalloc(&c->warm_count, 1));
      HIPCHK(c, hipMemsetAsync(c->warm_count, 0, sizeof(int), c->st));
    }
    ddk::launch_warm_apply(p, c->warm_given, c->warm_given_rms, c->warm_count, c->st);
    HIPCHK(c, hipGetLastError());
    c->warm_given = nullptr;
    c->n_warm_sweeps++;
  } else if (warm) {
    dd_status ws = warm_start(c, p);
    if (ws) return ws;
    c->n_warm_sweeps++;
  }
  c->warm_fresh[part] = 0;
  c->warm_level[part] = 0;
  ddk::launch_sweep_solve(r.dP, sc, r.ss, gr, kev);
  HIPCHK(c, hipGetLastError());
  ddk::launch_stats(r.dP, 1, r.dstats, c->st, kev ? kev + 2 * (DD_N_KERNELS - 1) : nullptr);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipEventRecord(r.ev1, c->st));
  HIPCHK(c, hipMemcpyAsync(r.hstats, r.dstats, sizeof(IterStatsDev), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  float ms = 0;
  hipEventElapsedTime(&ms, r.ev0, r.ev1);
  double mk[3 * DD_N_KERNELS];
  if (kev) runner_kernel_ms(r, mk);
  r.stream_prev = r.hstats[0].cells_bin[ddk::kNBins - 2];
  r.big_prev = r.hstats[0].cells_bin[ddk::kNBins - 1];
  return sweep_finish(c, part, r.hstats[0], ms, kev ? mk : nullptr, out);
}

// Gluing potential V on the cells of partition A of the current level
// (Sec. 6.3), solved on the device.  The graph: every ordered pair of basic
// cells of one B-cell is an oriented edge between their A-cells (the weight
// depends on the orientation, so both are taken).  Weights: log q(J1,J2) =
// log of the mu-mean of u_A/u_B over the first basic cell plus that of
// u_B/u_A over the second (one kernel, per basic cell).  V minimises
// sum_e (V(J2) - V(J1) - log q_e)^2 with mean zero: the sign follows the
// path-product form of the glued scalings, V(J2) - V(J1) ~ log q(J1,J2).
// The normal equations (graph Laplacian with edge counts as weights) are
// solved by conjugate gradients in one workgroup.  The host assembles only
// the geometry of the graph.
namespace {
struct GlueScratch {
  double *dq = nullptr, *work = nullptr, *ellw = nullptr, *deg = nullptr;
  int *ia = nullptr, *ib = nullptr, *incp = nullptr, *ince = nullptr, *elli = nullptr;
  int na = 0, ne = 0, max_it = 0, ellk = 0;
  ~GlueScratch() {
    dfree(dq);
    dfree(work);
    dfree(ellw);
    dfree(deg);
    dfree(ia);
    dfree(ib);
    dfree(incp);
    dfree(ince);
    dfree(elli);
  }
};
}  // namespace

constexpr double kGlueTol2 = 1e-24;  // squared relative residual of the CG solve
constexpr int kGlueMaxIt = 20000;

// Enqueue the solve on c->st: dV (na doubles) receives V, info[0..2] the CG
// steps and the final and initial squared residual norms.
static dd_status enqueue_glue(dd_ctx* c, GlueScratch& g, double* dV, double* info) {
  const Level& l = c->L[c->lev];
  const int nb = c->nb;
  const int na = c->cells[0].n;
  std::vector<int> cellA(nb, 0);
  for (int k = 0; k < na; k++) {
    const int4 t = c->cells[0].hq[k];
    const int ids[4] = {t.x, t.y, t.z, t.w};
    for (int a = 0; a < 4; a++)
      if (ids[a] >= 0) cellA[ids[a]] = k;
  }
  std::vector<int> e_ia, e_ib;
  for (int k = 0; k < c->cells[1].n; k++) {
    const int4 t = c->cells[1].hq[k];
    const int all[4] = {t.x, t.y, t.z, t.w};
    for (int a = 0; a < 4; a++)
      for (int b = 0; b < 4; b++)
        if (a != b && all[a] >= 0 && all[b] >= 0) {
          e_ia.push_back(all[a]);
          e_ib.push_back(all[b]);
        }
  }
  const int ne = (int)e_ia.size();
  std::vector<int> inc_ptr(na + 1, 0), inc_e(2 * (size_t)ne);
  for (int e = 0; e < ne; e++) {
    inc_ptr[cellA[e_ia[e]] + 1]++;
    inc_ptr[cellA[e_ib[e]] + 1]++;
  }
  for (int J = 0; J < na; J++) inc_ptr[J + 1] += inc_ptr[J];
  std::vector<std::vector<int>> nbr(na);
  {
    std::vector<int> fill(inc_ptr.begin(), inc_ptr.end() - 1);
    for (int e = 0; e < ne; e++) {
      const int Ja = cellA[e_ia[e]], Jb = cellA[e_ib[e]];
      inc_e[fill[Ja]++] = e << 1;
      inc_e[fill[Jb]++] = (e << 1) | 1;
      nbr[Ja].push_back(Jb);
      nbr[Jb].push_back(Ja);
    }
  }
  std::vector<int> adj_ptr(na + 1, 0), adj_idx;
  std::vector<double> adj_w, deg(na, 0.0);
  for (int J = 0; J < na; J++) {
    auto& v = nbr[J];
    std::sort(v.begin(), v.end());
    for (size_t k = 0; k < v.size();) {
      size_t m = k;
      while (m < v.size() && v[m] == v[k]) m++;
      adj_idx.push_back(v[k]);
      adj_w.push_back((double)(m - k));
      deg[J] += (double)(m - k);
      k = m;
    }
    adj_ptr[J + 1] = (int)adj_idx.size();
  }
  // the neighbour lists in ELL form (entry k of row J at k*na + J, the CSR
  // order kept, rows padded to a multiple of 8 with weight 0 on the row itself)
  // so that the Laplacian product issues every load of a row at once
  int kmax = 0;
  for (int J = 0; J < na; J++) kmax = std::max(kmax, adj_ptr[J + 1] - adj_ptr[J]);
  const int ellk = std::max(8, (kmax + 7) / 8 * 8);
  std::vector<int> ell_idx((size_t)ellk * na);
  std::vector<double> ell_w((size_t)ellk * na, 0.0);
  for (int J = 0; J < na; J++)
    for (int k = 0; k < ellk; k++) {
      const int q = adj_ptr[J] + k;
      const bool in = q < adj_ptr[J + 1];
      ell_idx[(size_t)k * na + J] = in ? adj_idx[q] : J;
      ell_w[(size_t)k * na + J] = in ? adj_w[q] : 0.0;
    }
  g.na = na;
  g.ne = ne;
  g.ellk = ellk;
  g.max_it = std::min(20 * na + 100, kGlueMaxIt);
  if (dmalloc(&g.dq, 2 * (size_t)nb) || dmalloc(&g.work, 4 * (size_t)na + 4) ||
      dmalloc(&g.ellw, (size_t)ellk * na + 1) || dmalloc(&g.deg, (size_t)na) ||
      dmalloc(&g.ia, (size_t)ne + 1) || dmalloc(&g.ib, (size_t)ne + 1) ||
      dmalloc(&g.incp, (size_t)na + 1) || dmalloc(&g.ince, 2 * (size_t)ne + 1) ||
      dmalloc(&g.elli, (size_t)ellk * na + 1))
    return fail(c, DD_ENOMEM, "gluing scratch");
  hipError_t e = hipSuccess;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (e == hipSuccess && bytes > 0)
      e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->st);
  };
  up(g.ia, e_ia.data(), sizeof(int) * ne);
  up(g.ib, e_ib.data(), sizeof(int) * ne);
  up(g.incp, inc_ptr.data(), sizeof(int) * (na + 1));
  up(g.ince, inc_e.data(), sizeof(int) * 2 * (size_t)ne);
  up(g.elli, ell_idx.data(), sizeof(int) * ell_idx.size());
  up(g.ellw, ell_w.data(), sizeof(double) * ell_w.size());
  up(g.deg, deg.data(), sizeof(double) * na);
  if (e != hipSuccess) return fail(c, DD_EHIP, "gluing upload: %s", hipGetErrorString(e));
  ddk::RefineParams R{};
  R.s = c->s;
  R.Hc = l.H;
  R.Wc = l.W;
  R.bwc = l.bw;
  R.eps = c->eps;
  R.mu_c = l.mu;
  R.alpha_a_c = c->alpha[0];
  R.alpha_b_c = c->alpha[1];
  ddk::launch_glue_ratios(R, g.dq, c->st);
  ddk::launch_cert_glue(g.incp, g.ince, g.ia, g.ib, g.dq, g.elli, g.ellw, g.ellk, g.deg, na,
                        g.max_it, kGlueTol2, g.work, dV, info, c->st);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(c, DD_EHIP, "gluing launch: %s", hipGetErrorString(e));
  return DD_OK;
}

__global__ void k_glue_apply(const double* aA, const double* V, double eps, int s, int Hc, int Wc,
                             double* out) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)Hc * Wc) return;
  const int r = (int)(i / Wc), cc = (int)(i % Wc);
  const int na_c = Wc / (2 * s);
  out[i] = aA[i] + eps * V[(r / (2 * s)) * na_c + cc / (2 * s)];
}

extern "C" dd_status dd_refine(dd_ctx* c) {
  if (!c) return DD_EINVAL;
  if (c->lev >= c->nlev - 1) return fail(c, DD_ESTATE, "already on the finest level");
  const Level& lc = c->L[c->lev];
  const Level& lf = c->L[c->lev + 1];
  ddk::RefineParams R{};
  R.s = c->s;
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
  // 1. gluing potential of the A-cells (device), glued coarse potential
  double *dV = nullptr, *fg = nullptr, *dinfo = nullptr;
  HIPCHK(c, dmalloc(&dV, (size_t)c->cells[0].n));
  HIPCHK(c, dmalloc(&fg, (size_t)lc.H * lc.W));
  HIPCHK(c, dmalloc(&dinfo, 4));
  {
    GlueScratch gs;
    dd_status gst = enqueue_glue(c, gs, dV, dinfo);
    if (gst != DD_OK) {
      dfree(dV);
      dfree(fg);
      dfree(dinfo);
      return gst;
    }
    long long n = (long long)lc.H * lc.W;
    hipLaunchKernelGGL(k_glue_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->st,
                       c->alpha[0], dV, c->eps, c->s, lc.H, lc.W, fg);
    double hinfo[3] = {0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(hinfo, dinfo, sizeof hinfo, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));  // the scratch of gs is released after this
    c->refine_glue_iters = (int)hinfo[0];
    c->refine_glue_resid = hinfo[2] > 0 ? std::sqrt(hinfo[1] / hinfo[2]) : 0.0;
  }
  dfree(dinfo);
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
  dfree(dV);
  dfree(fg);
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
  c->run.big_prev = -1;
  c->nb = nbf;
  c->last_part = -1;
  c->warm_fresh[0] = c->warm_fresh[1] = 1;
  c->warm_level[0] = c->warm_level[1] = 1;
  return upload_cells(c);
}

extern "C" dd_status dd_run_schedule(dd_ctx* c, dd_run_stats* out) {
  if (!c) return DD_EINVAL;
  if (c->in_batch) return fail(c, DD_ESTATE, "the context belongs to a batch");
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
      rs.newton_evals += it.newton_evals;
      rs.newton_mfma_flops += it.newton_mfma_flops;
      rs.newton_launches += ddk::kNDeferGroups;
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

// The diagnostics of dd_cost with the given scratch (H*W + 3*kDiagBlocks
// doubles on the context's device).
static dd_status cost_report(dd_ctx* c, double* scratch, dd_cost_report* r) {
  const Level& l = c->L[c->lev];
  ddk::launch_diag(c->row_off, c->row_len, c->col, c->val, l.mu, l.nu, c->s, l.H, l.W, l.bw, c->nb,
                   scratch, c->dscal, c->st);
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
    r->eps = c->last_eps;
    r->cost = c->last.cost;
    r->obj = c->last.obj;
    r->err_x = c->last.err_x;
  }
  return DD_OK;
}

extern "C" dd_status dd_cost(dd_ctx* c, dd_cost_report* r) {
  if (!c || !r) return DD_EINVAL;
  const Level& l = c->L[c->lev];
  dd_status s = ensure_px(c, (int64_t)l.H * l.W + 3 * ddk::kDiagBlocks);
  if (s) return s;
  return cost_report(c, c->px_scratch, r);
}

extern "C" dd_status dd_cost_noalloc(dd_ctx* c, dd_cost_report* r) {
  if (!c || !r) return DD_EINVAL;
  const Level& l = c->L[c->lev];
  const int64_t npx = (int64_t)l.H * l.W;
  if (npx > kNoAllocMaxPx)
    return fail(c, DD_ECAPACITY,
                "dd_cost_noalloc: level %d has %lld pixels, more than the %lld its static "
                "scratch holds (dd_cost has no such limit)",
                c->lev, (long long)npx, (long long)kNoAllocMaxPx);
  if (!c->noalloc_scratch) return fail(c, DD_ESTATE, "dd_cost_noalloc: scratch not set up");
  return cost_report(c, c->noalloc_scratch, r);
}

extern "C" dd_status dd_certificate(dd_ctx* c, dd_cert_report* r, double* alpha_hat,
                                   double* beta_hat) {
  if (!c || !r) return DD_EINVAL;
  if (c->last_part < 0) return fail(c, DD_ESTATE, "no half-iteration on this level yet");
  if (c->eps != c->last_eps)
    return fail(c, DD_ESTATE, "eps changed after the last half-iteration (%g -> %g)",
                c->last_eps, c->eps);
  const Level& l = c->L[c->lev];
  const int nb = c->nb;
  const long long npx = (long long)l.H * l.W;
  double *dV = nullptr, *ah = nullptr, *bh = nullptr, *scr = nullptr, *sums = nullptr;
  auto release = [&]() {
    dfree(dV);
    dfree(ah);
    dfree(bh);
    dfree(scr);
    dfree(sums);
  };
  if (dmalloc(&dV, (size_t)c->cells[0].n) || dmalloc(&ah, (size_t)npx) ||
      dmalloc(&bh, (size_t)npx) || dmalloc(&scr, 2 * (size_t)npx) || dmalloc(&sums, 8)) {
    release();
    return fail(c, DD_ENOMEM, "certificate scratch");
  }
  double hs[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  GlueScratch gs;
  // 1-2. overlap means and the least-squares potential V on the device
  dd_status gst = enqueue_glue(c, gs, dV, sums + 4);
  if (gst != DD_OK) {
    release();
    return gst;
  }
  // 3. glued potential; 4. Y-iteration over the stored support and the sums
  hipLaunchKernelGGL(k_glue_apply, dim3((unsigned)((npx + 255) / 256)), dim3(256), 0, c->st,
                     c->alpha[0], dV, c->eps, c->s, l.H, l.W, ah);
  ddk::launch_cert_y(c->row_off, c->row_len, c->col, ah, l.mu, l.nu, l.H, l.W, c->s, l.bw, nb, c->eps,
                     l.h, 0.5 * c->opt.cost_p, scr, bh, sums, c->st);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hs, sums, sizeof hs, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess && alpha_hat)
    e = hipMemcpyAsync(alpha_hat, ah, sizeof(double) * npx, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess && beta_hat)
    e = hipMemcpyAsync(beta_hat, bh, sizeof(double) * npx, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  release();
  if (e != hipSuccess) return fail(c, DD_EHIP, "certificate: %s", hipGetErrorString(e));
  memset(r, 0, sizeof(*r));
  r->primal = c->last.obj / c->eps;
  r->dual = (hs[0] + hs[1]) / c->eps - hs[2];
  r->gap = r->primal - r->dual;
  r->rel_gap = r->gap / r->primal;
  r->sum_nu = hs[2];
  r->n_uncovered = (int64_t)hs[3];
  r->n_edges = gs.ne;
  r->level = c->lev;
  r->eps = c->eps;
  r->cg_iters = (int)hs[4];
  r->cg_rel_resid = hs[6] > 0 ? std::sqrt(hs[5] / hs[6]) : 0.0;
  // the step cap reached before the residual bound: V is not the least-squares
  // solution and the dual is a bound for a less good candidate
  if (r->cg_iters >= gs.max_it && hs[5] > kGlueTol2 * hs[6]) return DD_ENOTCONV;
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
  dfree(rp);
  dfree(col);
  dfree(val);
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
  dfree(rp);
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

// ------------------------------------------------------------ batches

namespace {

// What a captured sweep depends on besides the parameter array's contents.
struct GraphKey {
  int n_prob = 0, total = 0, max_cells = 0, cap = 0, stream_wgs = 0, solver_pc = 0, newton_pc = 0,
      stream_max = 0, wg_cells = 0, quad = 0;
  const void* ptr[7] = {};
  bool operator==(const GraphKey& o) const {
    if (n_prob != o.n_prob || total != o.total || max_cells != o.max_cells || cap != o.cap ||
        stream_wgs != o.stream_wgs || solver_pc != o.solver_pc || newton_pc != o.newton_pc ||
        stream_max != o.stream_max || wg_cells != o.wg_cells || quad != o.quad)
      return false;
    for (int i = 0; i < 7; i++)
      if (ptr[i] != o.ptr[i]) return false;
    return true;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  long long last_use = 0;
};

constexpr size_t kGraphCache = 8;  // captured sweep shapes kept (A and B of a few levels)

// Position of a problem in its schedule.
struct SchedCursor {
  size_t stage = 0;
  int k = 0;            // sweeps done in the stage
  bool begun = false;   // the stage's refinements and eps change are applied
};

}  // namespace

struct dd_batch {
  std::string err;
  std::vector<dd_ctx*> cs;
  int flags = 0;
  // The batched launches run on a stream of the batch (a capturable one,
  // whatever the contexts' stream is), ordered with the contexts' stream
  // through events at the start and the end of every sweep.
  hipStream_t user_st = nullptr;
  hipStream_t own_st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  Runner run;
  long long n_sweeps = 0;
  int n_captures = 0;
  std::vector<GraphEntry> graphs;
  std::vector<SchedCursor> cur;  // schedule positions (dd_batch_schedule_step)
  bool cur_set = false;
};

static dd_status bfail(dd_batch* b, dd_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  b->err = buf;
  return s;
}

#define BHIPCHK(b, x)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      return bfail((b), e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EHIP, "%s: %s (%s:%d)", \
                   #x, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

static void drop_graph(GraphEntry& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

// One sweep over the problems with parts[i] >= 0 (partition of problem i).
static dd_status batch_sweep(dd_batch* b, const int* parts, dd_iter_stats* out) {
  Runner& r = b->run;
  const int n = (int)b->cs.size();
  std::vector<int> act;
  std::vector<HalfParams> hp;
  int total = 0, mx = 0;
  for (int i = 0; i < n; i++) {
    if (parts[i] < 0) continue;
    dd_ctx* c = b->cs[i];
    HalfParams p;
    const dd_status s = sweep_begin(c, parts[i], false, &p);
    if (s) return bfail(b, s, "problem %d: %s", i, c->err.c_str());
    act.push_back(i);
    hp.push_back(p);
    total += p.n_cells;
    mx = std::max(mx, p.n_cells);
  }
  const int na = (int)act.size();
  if (na == 0) return DD_OK;
  BHIPCHK(b, hipEventRecord(b->ev_in, b->user_st));
  BHIPCHK(b, hipStreamWaitEvent(r.main, b->ev_in, 0));
  BHIPCHK(b, runner_reserve(r, na, total));
  BHIPCHK(b, runner_stream(r, total));
  memcpy(r.hP, hp.data(), sizeof(HalfParams) * na);
  BHIPCHK(b, hipMemcpyAsync(r.dP, r.hP, sizeof(HalfParams) * na, hipMemcpyHostToDevice, r.main));
  bool all_quad = true;
  for (int i = 0; i < na; i++) all_quad = all_quad && hp[i].half_p == 1.0;
  const ddk::SweepSched sc = runner_sched(r, na, all_quad);
  const ddk::SweepGrid gr = plan_grid(r, total, mx, na);
  const bool graph = (b->flags & DD_BATCH_GRAPH) != 0;
  hipEvent_t* kev = (!graph && r.timing) ? r.kev : nullptr;
  if (graph) {
    GraphKey key;
    key.n_prob = na;
    key.total = total;
    key.max_cells = mx;
    key.cap = r.cap;
    key.stream_wgs = r.stream_wgs;
    key.solver_pc = r.solver_per_cu;
    key.newton_pc = r.newton_per_cu;
    key.stream_max = stream_limit(r);
    key.wg_cells = r.wg_cells;
    key.quad = sc.quad;
    const void* ptrs[7] = {r.dP, r.dstats, r.bin_list, r.defer_list, r.stream_tile, r.stream_S,
                           r.stream_nu};
    for (int i = 0; i < 7; i++) key.ptr[i] = ptrs[i];
    GraphEntry* ge = nullptr;
    for (auto& g : b->graphs)
      if (g.exec && g.key == key) ge = &g;
    if (!ge) {
      // capture this shape, in place of the least recently used one when full
      if (b->graphs.size() < kGraphCache) {
        b->graphs.emplace_back();
        ge = &b->graphs.back();
      } else {
        ge = &b->graphs[0];
        for (auto& g : b->graphs)
          if (g.last_use < ge->last_use) ge = &g;
        drop_graph(*ge);
      }
      BHIPCHK(b, hipStreamBeginCapture(r.main, hipStreamCaptureModeThreadLocal));
      ddk::launch_sweep_prep(r.dP, sc, r.ss, gr, nullptr);
      ddk::launch_sweep_solve(r.dP, sc, r.ss, gr, nullptr);
      ddk::launch_stats(r.dP, na, r.dstats, r.main, nullptr);
      const hipError_t le = hipGetLastError();
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(r.main, &g);
      BHIPCHK(b, le);
      BHIPCHK(b, ce);
      ge->graph = g;
      BHIPCHK(b, hipGraphInstantiate(&ge->exec, g, nullptr, nullptr, 0));
      ge->key = key;
      b->n_captures++;
    }
    ge->last_use = b->n_sweeps;
    BHIPCHK(b, hipEventRecord(r.ev0, r.main));
    BHIPCHK(b, hipGraphLaunch(ge->exec, r.main));
  } else {
    BHIPCHK(b, hipEventRecord(r.ev0, r.main));
    ddk::launch_sweep_prep(r.dP, sc, r.ss, gr, kev);
    ddk::launch_sweep_solve(r.dP, sc, r.ss, gr, kev);
    BHIPCHK(b, hipGetLastError());
    ddk::launch_stats(r.dP, na, r.dstats, r.main, kev ? kev + 2 * (DD_N_KERNELS - 1) : nullptr);
  }
  BHIPCHK(b, hipGetLastError());
  BHIPCHK(b, hipEventRecord(r.ev1, r.main));
  BHIPCHK(b, hipMemcpyAsync(r.hstats, r.dstats, sizeof(IterStatsDev) * na, hipMemcpyDeviceToHost,
                            r.main));
  BHIPCHK(b, hipEventRecord(b->ev_out, r.main));
  BHIPCHK(b, hipStreamWaitEvent(b->user_st, b->ev_out, 0));
  BHIPCHK(b, hipStreamSynchronize(r.main));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, r.ev0, r.ev1);
  double mk[3 * DD_N_KERNELS];
  if (kev) runner_kernel_ms(r, mk);
  int sp = 0;
  dd_status worst = DD_OK;
  for (int k = 0; k < na; k++) {
    const int i = act[k];
    sp += r.hstats[k].cells_bin[ddk::kNBins - 2];
    const dd_status s = sweep_finish(b->cs[i], parts[i], r.hstats[k], ms, kev ? mk : nullptr,
                                     out ? &out[i] : nullptr);
    if (s < 0) return bfail(b, s, "problem %d: %s", i, b->cs[i]->err.c_str());
    if (s > 0) worst = s;
  }
  r.stream_prev = sp;
  b->n_sweeps++;
  return worst;
}

extern "C" dd_status dd_batch_create(dd_ctx* const* ctxs, int n, int flags, dd_batch** out) {
  if (!out) return DD_EINVAL;
  *out = nullptr;
  if (!ctxs || n < 1 || n > ddk::kMaxProblems || (flags & ~DD_BATCH_GRAPH)) return DD_EINVAL;
  for (int i = 0; i < n; i++) {
    if (!ctxs[i] || ctxs[i]->in_batch || ctxs[i]->st != ctxs[0]->st) return DD_EINVAL;
    for (int j = 0; j < i; j++)
      if (ctxs[j] == ctxs[i]) return DD_EINVAL;
  }
  dd_batch* b = new dd_batch();
  b->cs.assign(ctxs, ctxs + n);
  b->flags = flags;
  b->user_st = ctxs[0]->st;
  bool timing = true;
  for (int i = 0; i < n; i++) timing = timing && ctxs[i]->opt.timing;
  hipError_t e = hipStreamCreateWithFlags(&b->own_st, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) e = runner_init(b->run, b->own_st, timing);
  if (e != hipSuccess) {
    dd_batch_free(b);
    return DD_EHIP;
  }
  for (int i = 0; i < n; i++) ctxs[i]->in_batch = true;
  *out = b;
  return DD_OK;
}

extern "C" dd_status dd_batch_half_iterate(dd_batch* b, int part, dd_iter_stats* stats) {
  if (!b) return DD_EINVAL;
  if (part != 0 && part != 1) return bfail(b, DD_EINVAL, "partition must be 0 or 1");
  std::vector<int> parts(b->cs.size(), part);
  return batch_sweep(b, parts.data(), stats);
}

// Move a problem to its next pending sweep (applying stage transitions on
// the way); false when its schedule is over.
static dd_status sched_advance(dd_ctx* c, SchedCursor& cur, bool* pending) {
  *pending = false;
  while (cur.stage < c->sched.size()) {
    const dd_stage& sg = c->sched[cur.stage];
    if (!cur.begun) {
      while (c->lev < sg.level) {
        const dd_status s = dd_refine(c);
        if (s < 0) return s;
      }
      if (sg.level != c->lev)
        return fail(c, DD_ESTATE, "schedule level %d below current %d", sg.level, c->lev);
      dd_set_eps(c, sg.eps);
      cur.begun = true;
    }
    if (cur.k < sg.n_half_iters) {
      *pending = true;
      return DD_OK;
    }
    cur.stage++;
    cur.k = 0;
    cur.begun = false;
  }
  return DD_OK;
}

extern "C" dd_status dd_batch_schedule_step(dd_batch* b, dd_iter_stats* stats, int* n_active) {
  if (!b) return DD_EINVAL;
  const int n = (int)b->cs.size();
  if (!b->cur_set) {
    b->cur.assign(n, SchedCursor());
    for (int i = 0; i < n; i++) b->cur[i].stage = b->cs[i]->next_stage;
    b->cur_set = true;
  }
  std::vector<int> parts(n);
  int na = 0;
  for (int i = 0; i < n; i++) {
    bool pending = false;
    const dd_status s = sched_advance(b->cs[i], b->cur[i], &pending);
    if (s < 0) return bfail(b, s, "problem %d: %s", i, b->cs[i]->err.c_str());
    parts[i] = pending ? (b->cur[i].k & 1) : -1;
    na += pending;
    if (stats) memset(&stats[i], 0, sizeof(dd_iter_stats));
  }
  if (n_active) *n_active = na;
  dd_status s = DD_OK;
  if (na > 0) {
    s = batch_sweep(b, parts.data(), stats);
    if (s < 0) return s;
    for (int i = 0; i < n; i++)
      if (parts[i] >= 0) b->cur[i].k++;
  }
  for (int i = 0; i < n; i++) b->cs[i]->next_stage = b->cur[i].stage;
  return s;
}

extern "C" dd_status dd_batch_run_schedule(dd_batch* b, dd_run_stats* out) {
  if (!b) return DD_EINVAL;
  const int n = (int)b->cs.size();
  std::vector<dd_run_stats> rs(n);
  for (int i = 0; i < n; i++) memset(&rs[i], 0, sizeof(dd_run_stats));
  std::vector<dd_iter_stats> it(n);
  const auto t0 = std::chrono::steady_clock::now();
  dd_status worst = DD_OK;
  for (;;) {
    int na = 0;
    const dd_status s = dd_batch_schedule_step(b, it.data(), &na);
    if (s < 0) return s;
    if (na == 0) break;
    if (s > 0) worst = s;
    for (int i = 0; i < n; i++) {
      const dd_iter_stats& t = it[i];
      if (t.n_cells == 0) continue;  // not in this sweep
      dd_run_stats& r = rs[i];
      r.n_half_iters++;
      r.n_cell_solves += t.n_cells;
      r.loops_total += t.loops_total;
      r.entry_evals += t.entry_evals;
      r.newton_evals += t.newton_evals;
      r.newton_mfma_flops += t.newton_mfma_flops;
      r.newton_launches += ddk::kNDeferGroups;
      r.n_failed += t.n_failed;
      r.n_safeguard += t.n_safeguard;
      r.n_newton += t.n_newton;
      r.nnz_max = std::max(r.nnz_max, t.nnz);
      for (int k = 0; k < DD_N_KERNELS; k++) r.ms_kernel[k] += t.ms_kernel[k];
      for (int k = 0; k < DD_N_BINS; k++) {
        r.launches_bin[k] += 1;
        r.evals_bin[k] += t.evals_bin[k];
      }
    }
  }
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (out)
    for (int i = 0; i < n; i++) {
      out[i] = rs[i];
      out[i].ms_total = ms;
    }
  return worst;
}

extern "C" dd_status dd_batch_info(const dd_batch* b, int* n_problems, long long* n_sweeps,
                                   int* n_captures) {
  if (!b) return DD_EINVAL;
  if (n_problems) *n_problems = (int)b->cs.size();
  if (n_sweeps) *n_sweeps = b->n_sweeps;
  if (n_captures) *n_captures = b->n_captures;
  return DD_OK;
}

extern "C" void dd_batch_free(dd_batch* b) {
  if (!b) return;
  if (b->own_st) (void)hipStreamSynchronize(b->own_st);
  for (auto& g : b->graphs) drop_graph(g);
  runner_free(b->run);
  if (b->own_st) (void)hipStreamDestroy(b->own_st);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  for (dd_ctx* c : b->cs) c->in_batch = false;
  delete b;
}

extern "C" const char* dd_batch_last_error(const dd_batch* b) {
  return b ? b->err.c_str() : "batch is NULL";
}

// ------------------------------------------------------------ launch tuning

namespace {

// Device copy of the state a sweep of one partition changes (the basic-cell
// rows and that partition's potentials), so that the sweep can be run again
// from the same state.
struct Snapshot {
  int64_t* row_off = nullptr;
  int* row_len = nullptr;
  int* col = nullptr;
  double* val = nullptr;
  double* alpha = nullptr;
  int64_t capE = 0, npx = 0, nnz = 0;
  int nb = 0, part = 0, last_part = -1;
  dd_iter_stats last{};
  double last_eps = 0;
  bool prev_valid = false;
  int warm_fresh[2] = {1, 1};
  int warm_level[2] = {1, 1};
  int n_warm_sweeps = 0;
};

const int kTuneSolver[] = {2, 4, 8, 16};
const int kTuneNewton[] = {1, 2, 4};
const int kTuneStream[] = {32, 64, 128, 256, 0};  // 0: two per compute unit
const int kTuneCells[] = {0, 1, 2, 4};             // 0: persistent workgroups

}  // namespace

static void snap_free(Snapshot& s) {
  (void)dfree(s.row_off);
  (void)dfree(s.row_len);
  (void)dfree(s.col);
  (void)dfree(s.val);
  (void)dfree(s.alpha);
  s = Snapshot();
}

static dd_status snap_take(dd_ctx* c, int part, Snapshot& s) {
  const Level& l = c->L[c->lev];
  s.nb = c->nb;
  s.capE = c->capE;
  s.npx = (int64_t)l.H * l.W;
  s.nnz = c->nnz;
  s.part = part;
  s.last_part = c->last_part;
  s.last = c->last;
  s.last_eps = c->last_eps;
  s.prev_valid = c->prev_valid;
  s.warm_fresh[0] = c->warm_fresh[0];
  s.warm_fresh[1] = c->warm_fresh[1];
  s.warm_level[0] = c->warm_level[0];
  s.warm_level[1] = c->warm_level[1];
  s.n_warm_sweeps = c->n_warm_sweeps;
  HIPCHK(c, dmalloc(&s.row_off, s.nb));
  HIPCHK(c, dmalloc(&s.row_len, s.nb));
  HIPCHK(c, dmalloc(&s.col, s.capE));
  HIPCHK(c, dmalloc(&s.val, s.capE));
  HIPCHK(c, dmalloc(&s.alpha, s.npx));
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  HIPCHK(c, hipMemcpyAsync(s.row_off, c->row_off, sizeof(int64_t) * s.nb, k, c->st));
  HIPCHK(c, hipMemcpyAsync(s.row_len, c->row_len, sizeof(int) * s.nb, k, c->st));
  HIPCHK(c, hipMemcpyAsync(s.col, c->col, sizeof(int) * s.capE, k, c->st));
  HIPCHK(c, hipMemcpyAsync(s.val, c->val, sizeof(double) * s.capE, k, c->st));
  HIPCHK(c, hipMemcpyAsync(s.alpha, c->alpha[part], sizeof(double) * s.npx, k, c->st));
  return DD_OK;
}

// The entry buffer may have grown since the snapshot (never shrunk), so the
// rows, which point below s.capE, stay valid.
static dd_status snap_restore(dd_ctx* c, const Snapshot& s) {
  if (c->capE < s.capE || c->nb != s.nb) return fail(c, DD_ESTATE, "state changed shape");
  const hipMemcpyKind k = hipMemcpyDeviceToDevice;
  HIPCHK(c, hipMemcpyAsync(c->row_off, s.row_off, sizeof(int64_t) * s.nb, k, c->st));
  HIPCHK(c, hipMemcpyAsync(c->row_len, s.row_len, sizeof(int) * s.nb, k, c->st));
  HIPCHK(c, hipMemcpyAsync(c->col, s.col, sizeof(int) * s.capE, k, c->st));
  HIPCHK(c, hipMemcpyAsync(c->val, s.val, sizeof(double) * s.capE, k, c->st));
  HIPCHK(c, hipMemcpyAsync(c->alpha[s.part], s.alpha, sizeof(double) * s.npx, k, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->nnz = s.nnz;
  c->last_part = s.last_part;
  c->last = s.last;
  c->last_eps = s.last_eps;
  c->prev_valid = s.prev_valid;
  c->warm_fresh[0] = s.warm_fresh[0];
  c->warm_fresh[1] = s.warm_fresh[1];
  c->warm_level[0] = s.warm_level[0];
  c->warm_level[1] = s.warm_level[1];
  c->n_warm_sweeps = s.n_warm_sweeps;
  return DD_OK;
}

static bool valid_launch(const dd_tune_point* t) {
  return t && t->solver_per_cu >= 1 && t->solver_per_cu <= 64 && t->newton_per_cu >= 1 &&
         t->newton_per_cu <= 16 && t->stream_wgs >= 0 && t->stream_wgs <= 4096 &&
         t->cells_per_wg >= 0 && t->cells_per_wg <= 1 << 20;
}

static void apply_launch(Runner& r, const dd_tune_point& t) {
  r.solver_per_cu = t.solver_per_cu;
  r.newton_per_cu = t.newton_per_cu;
  r.stream_max = t.stream_wgs;
  r.wg_cells = t.cells_per_wg;
}

static dd_tune_point launch_of(const Runner& r) {
  return dd_tune_point{r.solver_per_cu, r.newton_per_cu, r.stream_max, r.wg_cells, 0.0};
}

extern "C" dd_status dd_set_launch(dd_ctx* c, const dd_tune_point* cfg) {
  if (!c) return DD_EINVAL;
  if (!valid_launch(cfg)) return fail(c, DD_EINVAL, "launch sizes out of range");
  apply_launch(c->run, *cfg);
  return DD_OK;
}

extern "C" dd_status dd_batch_set_launch(dd_batch* b, const dd_tune_point* cfg) {
  if (!b) return DD_EINVAL;
  if (!valid_launch(cfg)) return bfail(b, DD_EINVAL, "launch sizes out of range");
  apply_launch(b->run, *cfg);
  return DD_OK;
}

extern "C" dd_status dd_get_launch(const dd_ctx* c, dd_tune_point* out) {
  if (!c || !out) return DD_EINVAL;
  *out = launch_of(c->run);
  return DD_OK;
}

// Time candidate launch configurations on the same sweep (state restored
// before each run and at the end) and keep the fastest, one axis at a time
// with the others at the best so far: register-solver cells per workgroup,
// the streamed solver's workgroups, Newton and (for persistent workgroups)
// solver workgroups per compute unit.  sweep() runs the sweep and returns its
// status and GPU time.  Every configuration gives the same results.
template <typename Sweep, typename Restore>
static dd_status tune_loop(Runner& r, int reps, Sweep sweep, Restore restore, dd_tune_point* best,
                           dd_tune_point* tried, int max_tried, int* n_tried) {
  int nt = 0;
  std::vector<dd_tune_point> seen;
  auto same = [](const dd_tune_point& a, const dd_tune_point& b) {
    return a.solver_per_cu == b.solver_per_cu && a.newton_per_cu == b.newton_per_cu &&
           a.stream_wgs == b.stream_wgs && a.cells_per_wg == b.cells_per_wg;
  };
  dd_tune_point b = launch_of(r);
  b.ms = INFINITY;
  auto run = [&](dd_tune_point c) -> dd_status {
    for (const auto& q : seen)
      if (same(q, c)) {
        if (q.ms < b.ms) b = q;
        return DD_OK;
      }
    apply_launch(r, c);
    double mn = INFINITY;
    for (int k = 0; k < reps; k++) {
      double ms = 0;
      dd_status s = restore();
      if (s < 0) return s;
      s = sweep(&ms);
      if (s < 0) return s;
      mn = std::min(mn, ms);
    }
    c.ms = mn;
    seen.push_back(c);
    if (tried && nt < max_tried) tried[nt] = c;
    nt++;
    if (c.ms < b.ms) b = c;
    return DD_OK;
  };
  dd_status s;
  for (int v : kTuneCells) {
    dd_tune_point c = b;
    c.cells_per_wg = v;
    if ((s = run(c)) < 0) return s;
  }
  for (int v : kTuneStream) {
    dd_tune_point c = b;
    c.stream_wgs = v;
    if ((s = run(c)) < 0) return s;
  }
  for (int v : kTuneNewton) {
    dd_tune_point c = b;
    c.newton_per_cu = v;
    if ((s = run(c)) < 0) return s;
  }
  if (b.cells_per_wg == 0)
    for (int v : kTuneSolver) {
      dd_tune_point c = b;
      c.solver_per_cu = v;
      if ((s = run(c)) < 0) return s;
    }
  if ((s = restore()) < 0) return s;
  apply_launch(r, b);
  if (best) *best = b;
  if (n_tried) *n_tried = nt;
  return DD_OK;
}

extern "C" dd_status dd_autotune(dd_ctx* c, int part, int reps, dd_tune_point* best,
                                 dd_tune_point* tried, int max_tried, int* n_tried) {
  if (!c) return DD_EINVAL;
  if (part != 0 && part != 1) return fail(c, DD_EINVAL, "partition must be 0 or 1");
  if (reps < 1 || max_tried < 0) return fail(c, DD_EINVAL, "reps must be >= 1");
  if (c->in_batch) return fail(c, DD_ESTATE, "the context belongs to a batch");
  Snapshot snap;
  dd_status s = snap_take(c, part, snap);
  if (s == DD_OK) {
    auto sweep = [&](double* ms) {
      dd_iter_stats it;
      const dd_status st = dd_half_iterate(c, part, &it);
      *ms = it.ms;
      return st;
    };
    auto restore = [&]() { return snap_restore(c, snap); };
    s = tune_loop(c->run, reps, sweep, restore, best, tried, max_tried, n_tried);
  }
  snap_free(snap);
  return s;
}

extern "C" dd_status dd_batch_autotune(dd_batch* b, int part, int reps, dd_tune_point* best,
                                       dd_tune_point* tried, int max_tried, int* n_tried) {
  if (!b) return DD_EINVAL;
  if (part != 0 && part != 1) return bfail(b, DD_EINVAL, "partition must be 0 or 1");
  if (reps < 1 || max_tried < 0) return bfail(b, DD_EINVAL, "reps must be >= 1");
  const int n = (int)b->cs.size();
  std::vector<Snapshot> snaps(n);
  dd_status s = DD_OK;
  for (int i = 0; i < n && s == DD_OK; i++) {
    s = snap_take(b->cs[i], part, snaps[i]);
    if (s) s = bfail(b, s, "problem %d: %s", i, b->cs[i]->err.c_str());
  }
  if (s == DD_OK) {
    std::vector<int> parts(n, part);
    std::vector<dd_iter_stats> it(n);
    auto sweep = [&](double* ms) {
      const dd_status st = batch_sweep(b, parts.data(), it.data());
      *ms = it[0].ms;
      return st;
    };
    auto restore = [&]() {
      for (int i = 0; i < n; i++) {
        const dd_status st = snap_restore(b->cs[i], snaps[i]);
        if (st < 0) return bfail(b, st, "problem %d: %s", i, b->cs[i]->err.c_str());
      }
      return DD_OK;
    };
    s = tune_loop(b->run, reps, sweep, restore, best, tried, max_tried, n_tried);
  }
  for (auto& sn : snaps) snap_free(sn);
  return s;
}

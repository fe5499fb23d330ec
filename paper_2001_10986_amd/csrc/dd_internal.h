// Internal interface between the host runtime (dd_runtime.hip) and the
// gfx950 kernels (dd_kernels.hip).  Not part of the public C-ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddk {

constexpr int kS = 4;          // default basic cell edge in pixels (s = 2 is also supported)
constexpr int kCellPx = 64;    // a composite cell (2s x 2s pixels) sits in a virtual 8x8 block
constexpr int kNRegBins = 5;   // register-resident solver bins: 1,2,4,8,16 waves
constexpr int kRegMaxU = 1024; // largest Y-support kept in registers (16 waves x 64)
constexpr int kStreamSlabs = 8;                // streamed solver: unions of up to 8 x 1024 points
constexpr int kStreamMaxU = kStreamSlabs * 1024;  // (processed in slabs of 512, dd_kernels.hip)
constexpr size_t kStreamTileFloats = (size_t)kStreamMaxU * 64;  // tile buffer per workgroup
constexpr int kNBins = kNRegBins + 2;          // + streamed solver + log-domain solver
constexpr int kFeatIn = 768;                   // warm-start network input width
constexpr int kWarmMaxU = 8192;                // cells with larger unions keep the plain start
constexpr double kWarmScale = 16.0;            // network output unit: 16 lam (h^2/eps)

// Everything one sweep over one partition needs.  Device pointers.
struct HalfParams {
  int H, W, bh, bw;
  int s;                       // basic cell edge in pixels (2 or 4)
  int n_cells, n_basic;
  int part;
  double h, eps, lam;          // lam = h^p / eps (cost in units of eps per pixel^p)
  double half_p, hp;           // cost c = |x-y|^p: p/2 (1 for the quadratic cost) and h^p
  double err_tol, trunc;
  int max_iter, safeguard, accel;
  int cap0;                    // loop cap of the first solve (safeguard trigger), <= max_iter
  int newton_after;            // >0: hand a cell to Newton steps after this many loops
  int fp64;                    // 1: every cell on the log-domain solver, FP64 exponentials
  const double* mu;            // level mu, H*W
  const double* nu;            // level nu, H*W
  double* alpha;               // potentials f of partition `part`, H*W (in/out)
  const int4* cell_q;          // basic-cell id per virtual quadrant (row-major), -1 if absent
  const int2* cell_org;        // virtual pixel origin (row, col) of the 8x8 block
  int64_t* row_off;            // per basic cell: first entry (in/out)
  int* row_len;                // per basic cell: entry count (in/out)
  int* ent_col;                // entries: linear Y pixel index
  double* ent_val;             // entries: mass
  int64_t* cell_toff;          // per cell: offset of its union in the union buffer
  int* cell_U;                 // per cell: union size
  int64_t* cell_ooff;          // per cell: offset of its output region in the entry buffer
  int* bin_count;              // kNBins counters
  int* bin_list;               // kNBins * n_cells cell ids
  int* uni_key;                // union: keys
  double* uni_nu;              // union: nu_J
  double* uni_G;               // union: scratch Y potential (big-cell solver)
  double* r_cost;
  double* r_obj;
  double* r_err;
  int* r_loops;
  int* r_status;
  long long* r_evals;
  long long* r_nev;            // per cell handed to a Newton launch: support passes x |X_J| x U there
  long long* r_nmf;            // and the FP64 matrix-core flops of its W formations
  long long* misc;             // [0] nnz_in, [1] out entries, [2] bad-row flag
  double* defer_F;             // potentials of cells handed to Newton steps (units of eps),
                               // 64 per cell, indexed by cell
  long long capE;              // entry buffer capacity (rows are checked against it)
};

constexpr int kNDeferGroups = 4;  // Newton launches per sweep (one per stream)

// A sweep runs the cells of one or more problems (each with its own
// HalfParams, in a device array) through the same solver launches.  A work
// item names a problem and one of its cells.
constexpr int kItemShift = 21;
constexpr int kItemCellMask = (1 << kItemShift) - 1;
constexpr int kMaxProblems = 1 << (31 - kItemShift);
struct SweepSched {
  int n_prob;
  int cap;                     // items each bin list / Newton list can hold
  int* bin_count;              // kNBins: items per bin over all problems
  int* bin_list;               // kNBins * cap items, problem-major within a bin
  int* queue;                  // next item of each solver launch (kNBins + kNDeferGroups)
  int* defer_count;            // kNDeferGroups: items handed to Newton steps per group
  int* defer_list;             // kNDeferGroups * cap items
  float* stream_tile;          // streamed solver: kStreamTileFloats per workgroup
  float* stream_S;             // streamed solver: S(y), kStreamMaxU per workgroup
  float* stream_nu;            // streamed solver: nu_J(y) in FP32, kStreamMaxU per workgroup
  int stream_wgs;              // workgroups the streamed-solver buffers are sized for
  int wg_cells;                // register solvers: cells per workgroup (0: until the queue is empty)
  int quad;                    // 1: every problem of the sweep has the quadratic cost
};

// c(x,y) / h^p for pixel offsets (dr, dc): |d|^p with p = 2 half_p, a cost
// h(x - y) with h strictly convex (Sec. 7.1); exact in integers for the
// quadratic cost (half_p == 1, the paper's experiments).
__device__ __forceinline__ double cost_units(int dr, int dc, double half_p) {
  const int d2 = dr * dr + dc * dc;
  if (half_p == 1.0) return (double)d2;
  return d2 > 0 ? exp(half_p * log((double)d2)) : 0.0;
}

// Basic cell of pixel (i, j) of a composite cell's virtual 8x8 block: the
// cell covers rows and columns [0, 2s) of the block as a 2x2 arrangement of
// s x s basic cells (quadrant 2 * (i >= s) + (j >= s)); -1 outside it.
__device__ __forceinline__ int block_quadrant(int i, int j, int s) {
  if (i >= 2 * s || j >= 2 * s) return -1;
  return (i >= s ? 2 : 0) + (j >= s ? 1 : 0);
}

// The solvers are compiled twice: QUAD for sweeps whose problems all have the
// quadratic cost (integer |d|^2, no transcendental work), and a general
// instantiation that forms every cost through cost_units.
template <bool QUAD>
__device__ __forceinline__ double cost_q(int dr, int dc, double half_p) {
  if constexpr (QUAD)
    return (double)(dr * dr + dc * dc);
  else
    return cost_units(dr, dc, half_p);
}

struct IterStatsDev {
  double cost, obj, err;
  long long loops_total, evals, nnz;
  long long newton_evals, newton_mfma;  // work of the Newton launches (cells handed over)
  long long out_entries, bad_rows;  // entries the sweep wrote; rows found out of range
  int loops_max, n_failed, n_safeguard, n_newton, n_cells;
  long long evals_bin[kNBins];
  int cells_bin[kNBins];
};

// Streams of one sweep: the solver launches of the size bins run concurrently
// on `main` and three auxiliary streams (fork/join through events).
struct SweepStreams {
  hipStream_t main;
  hipStream_t aux[3];
  hipEvent_t fork;
  hipEvent_t join[3];
};
constexpr int kNKernels = 12;  // scan, union, scan_out, 5 register, streamed, big, newton, stats

constexpr int kNEvents = 2 * (kNKernels + kNDeferGroups - 1);

// Kernel launchers (all asynchronous).  ev: nullptr, or kNEvents events;
// ev[2k] and ev[2k+1] are recorded around kernel k on the stream it runs on;
// kernel 10 (Newton) is launched once per stream, the launches on the
// auxiliary streams take the slots kNKernels .. kNKernels + 2.
// Workgroups per solver launch (each loops over its bin's work queue).
struct SweepGrid {
  int bin[kNBins];   // solver launches of bins 0..kNBins-1
  int newton;        // the launch for the cells handed over to Newton steps
  int other;         // union kernel: workgroups per problem
};
// A sweep is prep (cell sizes, unions, per-problem bins, then the merged work
// lists) and solve (the concurrent solver launches and the Newton launches);
// a warm start may run in between.  P: device array of s.n_prob HalfParams.
void launch_sweep_prep(const HalfParams* P, const SweepSched& s, const SweepStreams& ss,
                       const SweepGrid& gr, hipEvent_t* ev);
void launch_sweep_solve(const HalfParams* P, const SweepSched& s, const SweepStreams& ss,
                        const SweepGrid& gr, hipEvent_t* ev);
// Per-problem statistics of the sweep: out[k] for problem k.
void launch_stats(const HalfParams* P, int n_prob, IterStatsDev* out, hipStream_t st,
                  hipEvent_t* ev2);
size_t sweep_max_static_lds();

void launch_validate(const double* mu, const double* nu, int s, int H, int W, double* out4,
                     hipStream_t st);
void launch_pyramid(const double* fine, double* coarse, int Hc, int Wc, hipStream_t st);
void launch_product_init(const int* ypos, int nzy, const double* nu, const double* bmass,
                         int n_basic, int* col, double* val, int64_t* row_off, int* row_len,
                         hipStream_t st);

// Diagnostics: out[0] = sum |sum_i nu_i - nu|, out[1] = sum_i | |nu_i| - |mu_i| |, out[2] = nnz.
// scratch_px holds H*W + 3*kDiagBlocks doubles.
constexpr int kDiagBlocks = 256;
void launch_diag(const int64_t* row_off, const int* row_len, const int* col, const double* val,
                 const double* mu, const double* nu, int s, int H, int W, int bw, int n_basic,
                 double* scratch_px, double* out3, hipStream_t st);

// Export: dense CSR from the gapped rows.
void launch_export(const int64_t* row_off, const int* row_len, const int* col, const double* val,
                   int n_basic, int64_t* row_ptr_dev, int* col_out, double* val_out,
                   hipStream_t st);
void launch_scan_rows(const int* row_len, int n, int64_t* row_ptr, hipStream_t st);

// Warm start: features of every cell (BF16 rows of kFeatIn, zero for cells
// above kWarmMaxU); then the network output applied to alpha.
void launch_warm_features(const HalfParams& p, unsigned short* X, hipStream_t st);
void launch_warm_apply(const HalfParams& p, const float* Y, float min_rms, int* n_applied,
                       hipStream_t st);
// Training samples of the last sweep (FP32 features from the potentials the
// sweep started from, targets = the solve's change of the potential, masks).
void launch_collect(const HalfParams& p, const double* alpha_prev, float* X, float* T, float* M,
                    int* ids, int cap, int* count, hipStream_t st);

// Refinement.
struct RefineParams {
  int s;                       // basic cell edge in pixels
  int Hc, Wc, bwc, Hf, Wf, bwf, n_basic_f;
  double eps;
  const double* mu_c; const double* nu_c; const double* mu_f; const double* nu_f;
  const double* alpha_a_c; const double* alpha_b_c;
  const int64_t* row_off_c; const int* row_len_c; const int* col_c; const double* val_c;
  int64_t* row_off_f; int* row_len_f; int* col_f; double* val_f;
};
void launch_refine_rows(const RefineParams& r, hipStream_t st);
// log q for every (A,B) overlap: per basic cell b: out[2b] = log mean_b exp((fA-fB)/eps),
// out[2b+1] = log mean_b exp((fB-fA)/eps) (mu-weighted)
void launch_glue_ratios(const RefineParams& r, double* out, hipStream_t st);
void launch_interp(const double* fglued_c, int Hc, int Wc, double* fa, double* fb, int Hf,
                   int Wf, hipStream_t st);

// Primal-dual certificate: beta_hat(y) = exact Y-iteration of alpha_hat over
// the stored support (-eps log sum_x exp((alpha_hat(x) - c(x,y))/eps) mu(x)),
// sums[0..3] = (sum alpha_hat mu, sum beta_hat nu, sum nu, uncovered pixels).
// scratch holds 2*H*W doubles; beta_hat H*W; sums 4.
// Gluing potential of the certificate on the device: right-hand side from the
// per-basic-cell overlap means q and the oriented edges (e_ia -> e_ib, basic
// cell ids; inc_* the edges incident to each A-cell, (edge << 1) | head), then
// conjugate gradients on the A-cell Laplacian (adj_* neighbours with edge
// counts, deg the diagonal) in one workgroup, mean zero.  work holds 4*na
// doubles; info[0..2] = (iterations, final r.r, initial r.r).
// ell_idx / ell_w: the neighbours of A-cell J and the edge counts at k*na + J,
// k < ell_k (a multiple of 8; padding: J itself with weight 0)
void launch_cert_glue(const int* inc_ptr, const int* inc_e, const int* e_ia, const int* e_ib,
                      const double* q, const int* ell_idx, const double* ell_w, int ell_k,
                      const double* deg, int na, int max_it, double tol2, double* work,
                      double* V, double* info, hipStream_t st);
void launch_cert_y(const int64_t* row_off, const int* row_len, const int* col,
                   const double* alpha_hat, const double* mu, const double* nu, int H, int W,
                   int bs, int bw, int n_basic, double eps, double h, double half_p,
                   double* scratch, double* beta_hat, double* sums, hipStream_t st);

// Single sparse multi-scale Sinkhorn (dd_single.hip).  dir 0: X side (p an X
// pixel, the other side Y), dir 1: Y side.
void sg_launch_support(int dir, const double* pot_p, const double* pot_q, int H, int W,
                       double hp, double half_p, double eps, double log_theta, int margin,
                       int4* box, long long* counts, hipStream_t st);
int sg_pass_blocks(int H, int W);
void sg_launch_pass(int dir, const double* pot_p, const double* pot_q, const double* m_p,
                    const double* m_q, double* scale_p, const double* scale_q, const int4* box,
                    int H, int W, double hp, double half_p, double eps, double log_theta,
                    int update, double* part, double* out5, hipStream_t st);
void sg_launch_absorb(double* pot, double* scale, const double* m, long long n, double eps,
                      hipStream_t st);
void sg_launch_fill_box(int4* box, long long n, int4 v, hipStream_t st);
void sg_launch_fill(double* a, long long n, double v, hipStream_t st);
void sg_launch_widen(int4* box, long long n, int H, int W, int margin, hipStream_t st);
void sg_launch_refine_box(const int4* cbox, int Wc, int4* fbox, int Hf, int Wf, int margin,
                          hipStream_t st);
void sg_launch_final(const double* alpha, const double* beta, const double* mu, const double* nu,
                     const double* u, const double* v, const int4* xbox, int H, int W, double hp,
                     double half_p, double eps, double log_theta, double* part, double* out5,
                     hipStream_t st);
void sg_launch_total(const double* pot, const double* scale, const double* m, long long n,
                     double eps, double* out, hipStream_t st);

}  // namespace ddk

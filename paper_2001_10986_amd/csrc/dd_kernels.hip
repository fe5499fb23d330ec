// gfx950 kernels of one domain-decomposition sweep (Algorithm 2 of Bonafini &
// Schmitzer) and of the coarse-to-fine refinement (Sec. 6.4).
//
// One sweep over a partition is, per composite cell J:
//   union    : Y_J = union of the supports of nu_i (i in J), nu_J = sum nu_i
//              (Algorithm 2, "compute Y-marginal on cell");
//   solve    : stabilised Sinkhorn between mu_J and nu_J from the stored
//              potential, stopped on the L1 X-marginal error after a
//              Y-iteration (Sec. 6.2);
//   split    : nu_i(y) = plan restricted to X_i x {y} (Algorithm 2, "extract
//              new basic partial marginals");
//   balance  : BalanceMeasures (Sec. 6.2), truncation (Sec. 6.1 (ii)) and
//              compaction into the basic-cell rows.
#include "dd_internal.h"

#include <float.h>
#include <math.h>
#include <algorithm>

namespace ddk {

#define DEVI __device__ __forceinline__

static constexpr double kLog2e = 1.4426950408889634;
static constexpr double kLn2 = 0.6931471805599453;
static constexpr float kLn2f = 0.6931471805599453f;

// ------------------------------------------------------------ primitives

DEVI void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

DEVI float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
DEVI float fast_log2(float x) { return __builtin_amdgcn_logf(x); }

template <typename T>
DEVI T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
DEVI T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}
template <typename T>
DEVI T wave_min(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u < v ? u : v;
  }
  return v;
}
// Wave-wide sums through DPP lane moves (a fixed tree: quad swaps, row
// rotations, row broadcasts; the total lands in lane 63 and is read back as a
// uniform value).  Cheaper than the LDS crossbar behind __shfl_xor.
template <int CTRL>
DEVI int dpp_mov0(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
DEVI double dpp_d(double v) {
  const long long q = __builtin_bit_cast(long long, v);
  const int lo = dpp_mov0<CTRL>((int)(q & 0xffffffffll));
  const int hi = dpp_mov0<CTRL>((int)(q >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
DEVI double wave_sum_dpp(double v) {
  v += dpp_d<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x124>(v);  // row_ror:4
  v += dpp_d<0x128>(v);  // row_ror:8
  v += dpp_d<0x142>(v);  // row_bcast:15
  v += dpp_d<0x143>(v);  // row_bcast:31
  const long long q = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(q & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(q >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

DEVI float wave_sum_dpp_f(float v) {
  v += __builtin_bit_cast(float, dpp_mov0<0xb1>(__builtin_bit_cast(int, v)));
  v += __builtin_bit_cast(float, dpp_mov0<0x4e>(__builtin_bit_cast(int, v)));
  v += __builtin_bit_cast(float, dpp_mov0<0x124>(__builtin_bit_cast(int, v)));
  v += __builtin_bit_cast(float, dpp_mov0<0x128>(__builtin_bit_cast(int, v)));
  v += __builtin_bit_cast(float, dpp_mov0<0x142>(__builtin_bit_cast(int, v)));
  v += __builtin_bit_cast(float, dpp_mov0<0x143>(__builtin_bit_cast(int, v)));
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

template <typename T>
DEVI T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Block exclusive scan of one value per thread; returns the prefix and the
// block total.  `sh` needs nwaves entries.  Contains barriers.
template <typename T>
DEVI T block_excl_scan(T v, T* sh, T* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  T inc = wave_incl_scan(v, lane);
  __syncthreads();
  if (lane == 63) sh[wave] = inc;
  __syncthreads();
  T off = 0, tot = 0;
  for (int w = 0; w < nw; w++) {
    T s = sh[w];
    if (w < wave) off += s;
    tot += s;
  }
  *total = tot;
  return off + inc - v;
}

// Deterministic block sum (fixed tree) of a double; result valid in all threads.
DEVI double block_sum_d(double v, double* sh) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < nw; w++) t += sh[w];
  return t;
}

DEVI void split_key(int key, int W, double invW, int* r, int* c) {
  int rr = (int)(((double)key + 0.5) * invW);
  *r = rr;
  *c = key - rr * W;
}

// ------------------------------------------------------------ scans over cells

// cell_toff = exclusive scan of T_J = sum of the row lengths of J's basic cells
__global__ __launch_bounds__(1024) void k_scan_T(const HalfParams* __restrict__ P) {
  __shared__ long long sh[16];
  const HalfParams& p = P[blockIdx.x];
  if (threadIdx.x == 0) p.misc[2] = 0;  // bad-row flag, raised by the union kernel
  long long carry = 0;
  for (int base = 0; base < p.n_cells; base += 1024) {
    int i = base + threadIdx.x;
    long long t = 0;
    if (i < p.n_cells) {
      int4 q = p.cell_q[i];
      if (q.x >= 0) t += p.row_len[q.x];
      if (q.y >= 0) t += p.row_len[q.y];
      if (q.z >= 0) t += p.row_len[q.z];
      if (q.w >= 0) t += p.row_len[q.w];
    }
    long long tot;
    long long ex = block_excl_scan(t, sh, &tot);
    if (i < p.n_cells) p.cell_toff[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) p.misc[0] = carry;
}

// Cells handed to Newton steps are collected per group of solver launches
// that share a stream, so that each group's Newton launch can follow its
// producers on that stream: bin 2 (main stream), bins 0 and 3, bins 1 and 4,
// and the streamed solver (bin 5).
DEVI int defer_group(int bin) {
  return bin == 2 ? 0 : bin == 0 || bin == 3 ? 1 : bin == 1 || bin == 4 ? 2 : 3;
}

// Size bin of a cell (the FP64 instantiation puts every cell on the
// log-domain solver).
DEVI int bin_of(int U);
DEVI int cell_bin(const HalfParams& p, int U);

DEVI int bin_of(int U) {
  if (U <= 64) return 0;
  if (U <= 128) return 1;
  if (U <= 256) return 2;
  if (U <= 512) return 3;
  if (U <= kRegMaxU) return 4;
  if (U <= kStreamMaxU) return 5;
  return 6;
}

DEVI int cell_bin(const HalfParams& p, int U) { return p.fp64 ? kNBins - 1 : bin_of(U); }

// cell_ooff = exclusive scan of |J| * U_J; stable lists of cells per size bin
__global__ __launch_bounds__(1024) void k_scan_out(const HalfParams* __restrict__ P) {
  const HalfParams& p = P[blockIdx.x];
  __shared__ long long sh[16];
  __shared__ int swc[16][kNBins];
  __shared__ int srun[kNBins];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x < kNBins) srun[threadIdx.x] = 0;
  long long carry = 0;
  for (int base = 0; base < p.n_cells; base += 1024) {
    int i = base + threadIdx.x;
    long long t = 0;
    int b = -1;
    if (i < p.n_cells) {
      int4 q = p.cell_q[i];
      int nq = (q.x >= 0) + (q.y >= 0) + (q.z >= 0) + (q.w >= 0);
      int U = p.cell_U[i];
      t = (long long)nq * U;
      b = cell_bin(p, U);
    }
    long long tot;
    long long ex = block_excl_scan(t, sh, &tot);
    if (i < p.n_cells) p.cell_ooff[i] = carry + ex;
    carry += tot;
    unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    unsigned long long mine = 0;
    for (int bb = 0; bb < kNBins; bb++) {
      unsigned long long m = __ballot(b == bb);
      if (lane == 0) swc[wave][bb] = __popcll(m);
      if (b == bb) mine = m;
    }
    __syncthreads();
    if (b >= 0) {
      int off = srun[b];
      for (int w = 0; w < wave; w++) off += swc[w][b];
      off += __popcll(mine & lt);
      p.bin_list[b * p.n_cells + off] = i;
    }
    __syncthreads();
    if (threadIdx.x < kNBins) {
      int s = 0;
      for (int w = 0; w < 16; w++) s += swc[w][threadIdx.x];
      srun[threadIdx.x] += s;
    }
    __syncthreads();
  }
  if (threadIdx.x < kNBins) p.bin_count[threadIdx.x] = srun[threadIdx.x];
  if (threadIdx.x == 0) p.misc[1] = carry;
}

// Work lists of the sweep: the per-problem bin lists concatenated in problem
// order (workgroup k copies problem k's items), and the launch counters
// cleared (a kernel rather than a memset, so that a captured graph holds no
// memset nodes).
__global__ __launch_bounds__(256) void k_sched(const HalfParams* __restrict__ P, SweepSched s) {
  const int k = blockIdx.x;
  const HalfParams& p = P[k];
  if (k == 0 && threadIdx.x < kNBins + kNDeferGroups) {
    s.queue[threadIdx.x] = 0;
    if (threadIdx.x < kNDeferGroups) s.defer_count[threadIdx.x] = 0;
  }
  for (int b = 0; b < kNBins; b++) {
    int off = 0, tot = 0;
    for (int j = 0; j < s.n_prob; j++) {
      const int c = P[j].bin_count[b];
      off += j < k ? c : 0;
      tot += c;
    }
    if (k == 0 && threadIdx.x == 0) s.bin_count[b] = tot;
    const int n = p.bin_count[b];
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      s.bin_list[(int64_t)b * s.cap + off + i] = (k << kItemShift) | p.bin_list[b * p.n_cells + i];
  }
}

// ------------------------------------------------------------ union (gather)

// Sorted union of up to four sorted rows and the summed masses.  The keys are
// marked in a bitmap over the 2D bounding box of the support (row-major, so
// bit order is key order), processed in bands of rows when the box is large;
// a popcount prefix gives every key its rank.  Masses of equal keys are summed
// in basic-cell order, so the result is deterministic.
constexpr int kUnionThreads = 256;
constexpr int kBitWords = 2048;  // 65536 bits per band

__global__ __launch_bounds__(kUnionThreads) void k_union(const HalfParams* __restrict__ P) {
  const HalfParams& p = P[blockIdx.y];
  __shared__ uint32_t bits[kBitWords];
  __shared__ int wpre[kBitWords];
  __shared__ int shi[8];
  __shared__ long long shl[8];
  const int tid = threadIdx.x;
  const double invW = 1.0 / p.W;
  for (int cell = blockIdx.x; cell < p.n_cells; cell += gridDim.x) {
    int4 q4 = p.cell_q[cell];
    int bq[4] = {q4.x, q4.y, q4.z, q4.w};
    int64_t off[4];
    int len[4], pre[5];
    int nr = 0;
    pre[0] = 0;
    for (int a = 0; a < 4; a++)
      if (bq[a] >= 0) {
        off[nr] = p.row_off[bq[a]];
        len[nr] = p.row_len[bq[a]];
        if (off[nr] < 0 || len[nr] < 0 || off[nr] + len[nr] > p.capE) {
          if (tid == 0) atomicOr((unsigned long long*)&p.misc[2], 1ull);
          len[nr] = 0;
          off[nr] = 0;
        }
        pre[nr + 1] = pre[nr] + len[nr];
        nr++;
      }
    const int T = pre[nr];
    const int64_t base = p.cell_toff[cell];
    if (T == 0) {
      if (tid == 0) p.cell_U[cell] = 0;
      continue;
    }
    int rmin = INT_MAX, rmax = -1;
    for (int a = 0; a < nr; a++)
      if (len[a] > 0) {
        int r0, c0, r1, c1;
        split_key(min(max(p.ent_col[off[a]], 0), p.H * p.W - 1), p.W, invW, &r0, &c0);
        split_key(min(max(p.ent_col[off[a] + len[a] - 1], 0), p.H * p.W - 1), p.W, invW, &r1, &c1);
        rmin = min(rmin, r0);
        rmax = max(rmax, r1);
      }
    int cmn = INT_MAX, cmx = -1;
    for (int e = tid; e < T; e += kUnionThreads) {
      int a = 0;
      while (e >= pre[a + 1]) a++;
      int r, c;
      split_key(p.ent_col[off[a] + (e - pre[a])], p.W, invW, &r, &c);
      cmn = min(cmn, c);
      cmx = max(cmx, c);
    }
    cmn = wave_min(cmn);
    cmx = wave_max(cmx);
    __syncthreads();
    if ((tid & 63) == 0) {
      shi[tid >> 6] = cmn;
      shi[4 + (tid >> 6)] = cmx;
    }
    __syncthreads();
    const int cmin = min(min(shi[0], shi[1]), min(shi[2], shi[3]));
    const int cmax = max(max(shi[4], shi[5]), max(shi[6], shi[7]));
    const int bwid = cmax - cmin + 1;
    const int rows_per_band = max(1, (kBitWords * 32) / bwid);
    int U = 0;
    for (int r0 = rmin; r0 <= rmax; r0 += rows_per_band) {
      const int r1 = min(rmax, r0 + rows_per_band - 1);
      const int nw = ((r1 - r0 + 1) * bwid + 31) >> 5;
      __syncthreads();
      for (int w = tid; w < nw; w += kUnionThreads) bits[w] = 0u;
      __syncthreads();
      for (int e = tid; e < T; e += kUnionThreads) {
        int a = 0;
        while (e >= pre[a + 1]) a++;
        int r, c;
        split_key(p.ent_col[off[a] + (e - pre[a])], p.W, invW, &r, &c);
        if (r >= r0 && r <= r1) {
          int b = (r - r0) * bwid + (c - cmin);
          atomicOr(&bits[b >> 5], 1u << (b & 31));
        }
      }
      __syncthreads();
      // exclusive popcount prefix over the band's words (8 words per thread)
      int loc = 0;
      const int w0 = tid * 8;
      for (int k = 0; k < 8; k++)
        if (w0 + k < nw) loc += __popc(bits[w0 + k]);
      long long tot;
      long long ex = block_excl_scan((long long)loc, shl, &tot);
      int run = (int)ex;
      for (int k = 0; k < 8; k++)
        if (w0 + k < nw) {
          wpre[w0 + k] = run;
          run += __popc(bits[w0 + k]);
        }
      const int cnt = (int)tot;
      for (int i = tid; i < cnt; i += kUnionThreads) p.uni_nu[base + U + i] = 0.0;
      __syncthreads();
      for (int a = 0; a < nr; a++) {
        for (int e = tid; e < len[a]; e += kUnionThreads) {
          int key = p.ent_col[off[a] + e];
          int r, c;
          split_key(key, p.W, invW, &r, &c);
          if (r >= r0 && r <= r1) {
            int b = (r - r0) * bwid + (c - cmin);
            uint32_t wd = bits[b >> 5];
            int pos = U + wpre[b >> 5] + __popc(wd & ((1u << (b & 31)) - 1u));
            p.uni_key[base + pos] = key;
            p.uni_nu[base + pos] += p.ent_val[off[a] + e];
          }
        }
        __syncthreads();
      }
      U += cnt;
    }
    if (tid == 0) p.cell_U[cell] = U;
    __syncthreads();
  }
}

// ------------------------------------------------------------ cell geometry

struct CellGeo {
  int R0, C0;      // virtual origin of the 8x8 block
  int bq[4];       // basic id per virtual quadrant or -1
  int nq;          // valid quadrants
  int qidx[4];     // index of the quadrant among the valid ones (segment number)
};

DEVI CellGeo load_geo(const HalfParams& p, int cell) {
  CellGeo g;
  int4 q = p.cell_q[cell];
  int2 o = p.cell_org[cell];
  g.R0 = o.x;
  g.C0 = o.y;
  g.bq[0] = q.x;
  g.bq[1] = q.y;
  g.bq[2] = q.z;
  g.bq[3] = q.w;
  g.nq = 0;
  for (int a = 0; a < 4; a++) {
    g.qidx[a] = g.bq[a] >= 0 ? g.nq : -1;
    if (g.bq[a] >= 0) g.nq++;
  }
  return g;
}

// Balancing, truncation and compaction of the basic marginals of one cell
// (BalanceMeasures of Sec. 6.2; truncation of Sec. 6.1 (ii)).  Each thread
// owns at most one support point y (index yi < U) and holds the four
// basic-cell values nq[0..3] for it.  READING (balance rule): with
// d_i = |mu_i| - |nu_i|, E = sum of -d_i over d_i < 0, D = sum of d_i over
// d_i > 0, T = min(E, D), every excess cell a loses the fraction
// T(-d_a)/(E |nu_a|) of its mass at every y and the freed mass R(y) goes to
// the deficit cells b in the proportions d_b/D.
struct CellOutSh {
  double red[16];
  long long scan[16];
  double dq[4], tq[4], E, D;
  long long cnt[4];
};

DEVI void balance_truncate_write(const HalfParams& p, const CellGeo& g, int64_t obase, int U,
                                 bool own, int yi, int key, double v[4], const double massmu[4],
                                 CellOutSh& sh) {
  // norms of the basic marginals
  double nrm[4];
#pragma unroll
  for (int a = 0; a < 4; a++) nrm[a] = block_sum_d(own ? v[a] : 0.0, sh.red);
  if (threadIdx.x == 0) {
    double E = 0, D = 0;
    for (int a = 0; a < 4; a++) {
      double d = g.bq[a] >= 0 ? massmu[a] - nrm[a] : 0.0;
      sh.dq[a] = d;
      if (d < 0) E += -d;
      if (d > 0) D += d;
    }
    double T = E < D ? E : D;
    for (int a = 0; a < 4; a++) sh.tq[a] = (T > 0 && sh.dq[a] < 0) ? T * (-sh.dq[a]) / (E * nrm[a]) : 0.0;
    sh.E = T > 0 ? E : 0.0;
    sh.D = T > 0 ? D : 0.0;
  }
  __syncthreads();
  if (own && sh.D > 0) {
    double R = 0;
    for (int a = 0; a < 4; a++)
      if (sh.dq[a] < 0 && g.bq[a] >= 0) {
        double r = v[a] * sh.tq[a];
        v[a] -= r;
        R += r;
      }
    for (int a = 0; a < 4; a++)
      if (sh.dq[a] > 0 && g.bq[a] >= 0) v[a] += R * sh.dq[a] / sh.D;
  }
  // truncation flags, packed 16 bits per quadrant
  unsigned long long flags = 0;
  if (own)
    for (int a = 0; a < 4; a++)
      if (g.bq[a] >= 0 && v[a] >= p.trunc && v[a] > 0.0) flags |= 1ull << (16 * a);
  // block scan (U may exceed the block size only in the big-cell solver,
  // which calls this once per chunk with a running carry in sh.cnt)
  long long tot;
  long long ex = block_excl_scan((long long)flags, sh.scan, &tot);
  if (own) {
    for (int a = 0; a < 4; a++)
      if ((flags >> (16 * a)) & 1ull) {
        long long pos = sh.cnt[a] + ((ex >> (16 * a)) & 0xffffll);
        if (pos < U) {
          int64_t at = obase + (int64_t)g.qidx[a] * U + pos;
          p.ent_col[at] = key;
          p.ent_val[at] = v[a];
        }
      }
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int a = 0; a < 4; a++) sh.cnt[a] += (tot >> (16 * a)) & 0xffffll;
  __syncthreads();
}

// Balancing, truncation and compaction for cells whose support exceeds the
// block size: the unbalanced split nu_J(y) S_i(y)/S(y) has been
// stashed at obase + qidx*U + yi; norms over the whole support, then the same
// BalanceMeasures rule, truncation and an order-preserving compaction chunk by
// chunk (out.cnt must be zero on entry).
DEVI void balance_compact_chunked(const HalfParams& p, const CellGeo& g, int64_t obase, int U,
                                  const double massmu[4], CellOutSh& out) {
  // balance: norms over the whole support, then per-y update and compaction
  double nrm[4];
  _Pragma("unroll") for (int a = 0; a < 4; a++) {
    double s = 0;
    if (g.bq[a] >= 0)
      for (int yi = (int)threadIdx.x; yi < U; yi += (int)blockDim.x) s += p.ent_val[obase + (int64_t)g.qidx[a] * U + yi];
    nrm[a] = block_sum_d(s, out.red);
  }
  if (threadIdx.x == 0) {
    double E = 0, D = 0;
    _Pragma("unroll") for (int a = 0; a < 4; a++) {
      double d = g.bq[a] >= 0 ? massmu[a] - nrm[a] : 0.0;
      out.dq[a] = d;
      if (d < 0) E += -d;
      if (d > 0) D += d;
    }
    double T = E < D ? E : D;
    _Pragma("unroll") for (int a = 0; a < 4; a++)
      out.tq[a] = (T > 0 && out.dq[a] < 0) ? T * (-out.dq[a]) / (E * nrm[a]) : 0.0;
    out.E = T > 0 ? E : 0.0;
    out.D = T > 0 ? D : 0.0;
  }
  __syncthreads();
  for (int y0 = 0; y0 < U; y0 += (int)blockDim.x) {
    const int yi = y0 + (int)threadIdx.x;
    const bool own = yi < U;
    double v[4] = {0, 0, 0, 0};
    int key = 0;
    if (own) {
      _Pragma("unroll") for (int a = 0; a < 4; a++)
        if (g.bq[a] >= 0) {
          const int64_t at = obase + (int64_t)g.qidx[a] * U + yi;
          v[a] = p.ent_val[at];
          key = p.ent_col[at];
        }
      if (out.D > 0) {
        double R = 0;
        _Pragma("unroll") for (int a = 0; a < 4; a++)
          if (g.bq[a] >= 0 && out.dq[a] < 0) {
            const double rr = v[a] * out.tq[a];
            v[a] -= rr;
            R += rr;
          }
        _Pragma("unroll") for (int a = 0; a < 4; a++)
          if (g.bq[a] >= 0 && out.dq[a] > 0) v[a] += R * out.dq[a] / out.D;
      }
    }
    unsigned long long flags = 0;
    if (own)
      _Pragma("unroll") for (int a = 0; a < 4; a++)
        if (g.bq[a] >= 0 && v[a] >= p.trunc && v[a] > 0.0) flags |= 1ull << (16 * a);
    long long tot;
    long long ex = block_excl_scan((long long)flags, out.scan, &tot);
    __syncthreads();  // every thread has read its chunk before any compacted write
    if (own)
      _Pragma("unroll") for (int a = 0; a < 4; a++)
        if ((flags >> (16 * a)) & 1ull) {
          const long long pos = out.cnt[a] + ((ex >> (16 * a)) & 0xffffll);
          if (pos < U) {
            const int64_t at = obase + (int64_t)g.qidx[a] * U + pos;
            p.ent_col[at] = key;
            p.ent_val[at] = v[a];
          }
        }
    __syncthreads();
    if (threadIdx.x == 0)
      _Pragma("unroll") for (int a = 0; a < 4; a++) out.cnt[a] += (tot >> (16 * a)) & 0xffffll;
    __syncthreads();
  }
}

// Chebyshev acceleration of the X-iteration (same rule as the oracle): one
// Sinkhorn loop F -> X(Y(F)) has a Jacobian with real eigenvalues in [0, rho)
// at the solution, so the Chebyshev semi-iteration for [0, rho] (Golub & Varga)
// converges at (1 - sqrt(1-rho))/(1 + sqrt(1-rho)).  The Y-iteration and the
// stopping test are untouched.  Every lane of the
// calling wave runs the rule on the same values, so the decision is uniform.
struct ChebState {
  double rho, omega;
  double sig2, gam, rmax;  // sigma^2, gamma and the abandon threshold of the current run
  double hist[17];
  int k, kstart, pstart, att;
};

DEVI void cheb_reset(ChebState& c) {
  c.rho = -1.0;
  c.omega = 1.0;
  c.k = 0;
  c.kstart = 0;
  c.pstart = 0;
  c.att = 0;
}

// returns true for an accelerated step F <- a F + b Fh + d Fprev.  Plain
// loops estimate rho from the error decay over the last 8 loops (at least 16
// plain loops after a (re)start); a Chebyshev run that decays slower than
// the square root of its promised rate over 16 loops is abandoned for plain
// loops; at most four runs per solve and rho <= 0.9999.  The constants of a
// run (sigma^2 = (rho/(2-rho))^2, gamma = 2/(2-rho), the threshold) are
// computed once when it starts, so an accelerated loop costs one division.
// Safe to run in every lane of a wave on the same state (same values written).
DEVI bool cheb_next(ChebState& c, int it, double err, double* a, double* b, double* d) {
  c.hist[it % 17] = err;
  if (c.rho < 0) {
    if (it - c.pstart >= 16 && c.att < 4) {
      const float r = fast_exp2(fast_log2((float)err / (float)c.hist[(it - 8) % 17]) * 0.125f);
      if (r > 0.8f) {
        const double rho = r < 0.9999f ? (double)r : 0.9999;
        const double sig = rho / (2 - rho), sq = sqrt(1 - rho);
        c.rho = rho;
        c.sig2 = sig * sig;
        c.gam = 2 / (2 - rho);
        c.rmax = sqrt((1 - sq) / (1 + sq));
        c.k = 0;
        c.kstart = it;
        c.att++;
      }
    }
    return false;
  }
  if (it - c.kstart >= 16 && (it - c.kstart) % 16 == 0) {
    const float robs = fast_exp2(fast_log2((float)err / (float)c.hist[(it - 16) % 17]) * 0.0625f);
    if (robs > c.rmax) {
      c.rho = -1;
      c.pstart = it;
      return false;
    }
  }
  if (c.k == 0)
    c.omega = 1;
  else if (c.k == 1)
    c.omega = 1 / (1 - c.sig2 / 2);
  else
    c.omega = 1 / (1 - c.sig2 * c.omega / 4);
  c.k++;
  *a = c.omega * (1 - c.gam);
  *b = c.omega * c.gam;
  *d = 1 - c.omega;
  return true;
}

// ------------------------------------------------------------ register solver

// Stabilised Sinkhorn for cells whose union fits NW*64 support points.
// Layout: a composite cell is a virtual 8x8 block of pixels x (absent pixels
// carry mu = 0).  Lane (wave w, xg = lane&7, yg = lane>>3) owns the 8 pixels
// of block row xg and the 8 support points y = w*64 + yg*8 + t, and keeps the
// 8x8 tile of the absorbed kernel
//     P(x,y) = exp(F0(x) + log mu(x) - C(x,y) - m(y)),  C = lam*|x-y|^2,
// in registers (m(y) = max_x of the exponent, so every column peaks at 1).
// The exponent is formed in FP64, the tile and the scaling iterations run in
// FP32, sums that decide stopping, masses and costs run in FP64.
//   Y-iteration:  S(y) = sum_x P(x,y) u(x),   w(y) = nu_J(y) / S(y)
//   X-marginal :  r(x) = sum_y P(x,y) w(y),   P_X pi(x) = u(x) r(x)
//   X-iteration:  u(x) = mu(x) / r(x)
// which is the Sinkhorn iteration of Remark "Sinkhorn algorithm" written in
// scalings relative to the absorbed potential F0 (plan pi = P u w).  When u
// leaves [e^-30, e^30] (or underflows) the X-iteration is done exactly in
// the log domain instead and F0 absorbs it (P is rebuilt).
template <int NW>
struct RegShared {
  double F0[64], Fmu[64], mu[64], F0orig[64], mx[64];
  float uw[NW][64];           // per-wave copy of the scaling u (every wave runs the X-update)
  float lupx[64];             // broadcast of the previous log2-scaling after an exact step
  float red[NW][512];         // per-wave transposition scratch (also FP64 scratch)
  float wred[2][NW][64];      // per-wave X partials, double-buffered by loop parity
  float w[NW * 64];           // w(y) = nu_J(y) / S(y)
  float nuf[NW * 64];
  int yrc[NW * 64];           // support point (row << 16 | col)
  ChebState cheb[NW];         // per-wave copy of the acceleration state
  int next;
  CellOutSh out;
};

// Transposition through the per-wave scratch: lane (yg, xg) provides v[t]
// for its 8 support points; returns, in lane (yg, xg), the sum over the 8
// lanes of its support group of v[t = xg], split into the block rows xg' < 4
// and xg' >= 4.  Element (yg, xg', t) lives at yg*64 + ((xg'^yg)&7)*8 + t:
// the xor swizzle spreads the 8 support groups over the LDS banks.
DEVI int tsw(int yg, int x, int t) { return yg * 64 + (((x ^ yg) & 7) << 3) + t; }

DEVI void transpose_y(float* rd, int xg, int yg, const float v[8], float* top, float* bot,
                      int split = 4) {
  wave_sync();
#pragma unroll
  for (int t = 0; t < 8; t++) rd[tsw(yg, xg, t)] = v[t];
  wave_sync();
  float a = 0.f, b = 0.f;
#pragma unroll
  for (int k = 0; k < 8; k++) {
    const float x = rd[tsw(yg, k, xg)];
    if (k < split) a += x; else b += x;
  }
  *top = a;
  *bot = b;
}

template <int CTRL>
DEVI float dpp_f(float v) {
  return __builtin_bit_cast(float, dpp_mov0<CTRL>(__builtin_bit_cast(int, v)));
}

// Sum over the 8 lanes of an 8-lane group (lane bits 0-2 = block row xg) of
// the per-lane partials v[t], t = 0..7: lane xg receives the total for t = xg.
// Recursive halving in registers (no LDS): half-row mirror (partner 7 - xg),
// quad mirror (partner with the other bit 1), quad swap (partner xg ^ 1);
// each step keeps the half of the values that the lane's bit selects.
DEVI float reduce8_t(const float v[8], int xg) {
  const bool b2 = (xg & 4) != 0, b1 = (xg & 2) != 0, b0 = (xg & 1) != 0;
  float a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const float send = b2 ? v[k] : v[4 + k];
    a[k] = (b2 ? v[4 + k] : v[k]) + dpp_f<0x141>(send);  // row_half_mirror
  }
#pragma unroll
  for (int m = 0; m < 2; m++) {
    const float send = b1 ? a[m] : a[2 + m];
    b[m] = (b1 ? a[2 + m] : a[m]) + dpp_f<0x1b>(send);  // quad_perm [3,2,1,0]
  }
  const float send = b0 ? b[0] : b[1];
  return (b0 ? b[1] : b[0]) + dpp_f<0xb1>(send);  // quad_perm [1,0,3,2]
}

// Sum over the 8 lanes that share a block row (lane bits 3-5 = yg) of the
// per-lane partials v[j], j = 0..7 (block columns): lane yg receives the total
// for j = yg.  Recursive halving: lane ^ 8 (row_ror:8 within a 16-lane row),
// then lane ^ 16 and lane ^ 32 (cross-row permutes).
DEVI float reduce8_j(const float v[8], int yg) {
  const bool c0 = (yg & 1) != 0, c1 = (yg & 2) != 0, c2 = (yg & 4) != 0;
  float a[4], b[2];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const float send = c0 ? v[2 * k] : v[2 * k + 1];
    a[k] = (c0 ? v[2 * k + 1] : v[2 * k]) + dpp_f<0x128>(send);  // row_ror:8
  }
#pragma unroll
  for (int m = 0; m < 2; m++) {
    const float send = c1 ? a[2 * m] : a[2 * m + 1];
    b[m] = (c1 ? a[2 * m + 1] : a[2 * m]) + __shfl_xor(send, 16, 64);
  }
  const float send = c2 ? b[0] : b[1];
  return (c2 ? b[1] : b[0]) + __shfl_xor(send, 32, 64);
}

DEVI double readlane0_d(double v) {
  const long long q = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(q & 0xffffffffll), 0);
  const int hi = __builtin_amdgcn_readlane((int)(q >> 32), 0);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// The X-update of one loop, run by every wave on the same data so that all
// waves take the same decisions without a second block barrier (lane = x):
// the X-marginal r = sum of the per-wave partials, the stopping error, the
// acceleration weights and the new scaling (written to this wave's copy).
struct XUpdate {
  float r;
  double err;
  bool go_on, flag, acc;
  double a, b, d;
};

DEVI XUpdate x_update(float r, double mu, float u, float* lup, float* unew_out, double tol,
                      int it, int max_iter, int accel, ChebState& cheb, int lane) {
  XUpdate o;
  o.r = r;
  // |u r - mu| per pixel (one rounding through the FMA) summed in FP32: 64
  // positive terms, relative error < 4e-6 of the sum, far below what the
  // stopping test resolves
  const float muf = (float)mu;
  const double e = (double)wave_sum_dpp_f(mu > 0 ? fabsf(fmaf(u, r, -muf)) : 0.f);
  o.err = e;
  o.go_on = !(e <= tol) && it < max_iter && (e == e);
  double a0 = 0, b0 = 1, d0 = 0;
  int acc0 = 0;
  if (lane == 0 && o.go_on && accel) acc0 = cheb_next(cheb, it, e, &a0, &b0, &d0);
  o.acc = __builtin_amdgcn_readlane(acc0, 0) != 0;
  o.a = readlane0_d(a0);
  o.b = readlane0_d(b0);
  o.d = readlane0_d(d0);
  const float un = mu > 0 ? muf * __builtin_amdgcn_rcpf(r) : 0.f;
  const float lu = mu > 0 ? fast_log2(u) : 0.f;
  float unew = un;
  if (o.acc && mu > 0) unew = fast_exp2((float)(o.a * lu + o.b * fast_log2(un) + o.d * *lup));
  const bool bad = mu > 0 && !(unew > 9.357623e-14f && unew < 1.0686475e13f && un > 0.f &&
                               un < 3.0e38f);
  const unsigned long long anyb = __ballot(bad);
  o.flag = o.go_on && anyb != 0ull;
  if (o.go_on && anyb == 0ull) {
    *unew_out = unew;
    *lup = lu;
  } else {
    *unew_out = u;
  }
  return o;
}

template <int NW, bool QUAD>
__global__ __launch_bounds__(NW * 64) void k_solve_reg(const HalfParams* __restrict__ P,
                                                       SweepSched s, int bin) {
  __shared__ RegShared<NW> sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int xg = lane & 7, yg = lane >> 3;
  const int ybase = wave * 64 + yg * 8;  // first of the lane's 8 support points
  const int count = s.bin_count[bin];
  float* rd = sh.red[wave];
  float* uw = sh.uw[wave];
  int taken = 0;
  for (;;) {
    // next item of this bin (a work queue, so that slow cells do not hold up
    // the cells behind them); with wg_cells > 0 a workgroup takes at most that
    // many cells and exits, so that launches on other streams get compute
    // units as this one's workgroups finish
    if (s.wg_cells > 0 && taken == s.wg_cells) break;
    taken++;
    if (tid == 0) sh.next = atomicAdd(&s.queue[bin], 1);
    __syncthreads();
    const int ci = sh.next;
    if (ci >= count) break;
    const int item = __builtin_amdgcn_readfirstlane(s.bin_list[(int64_t)bin * s.cap + ci]);
    const HalfParams& p = P[item >> kItemShift];
    const int cell = item & kItemCellMask;
    const double invW = 1.0 / p.W;
    const CellGeo g = load_geo(p, cell);
    const int U = p.cell_U[cell];
    const int64_t ub = p.cell_toff[cell];
    const int64_t obase = p.cell_ooff[cell];
    double* mbuf = p.uni_G + ub;  // m(y) of the absorbed tile, one per support point
    // ---- pixel data (pixel k = 8i + j of the block)
    if (tid < 64) {
      const int i = tid >> 3, j = tid & 7;
      const int qa = block_quadrant(i, j, p.s);
      const int bq = qa < 0 ? -1 : qa == 0 ? g.bq[0] : qa == 1 ? g.bq[1] : qa == 2 ? g.bq[2] : g.bq[3];
      const int r = g.R0 + i, c = g.C0 + j;
      double mu = 0, F0 = 0;
      if (bq >= 0) {
        mu = p.mu[(int64_t)r * p.W + c];
        F0 = p.alpha[(int64_t)r * p.W + c] / p.eps;
      }
      sh.mu[tid] = mu;
      sh.F0orig[tid] = F0;
      sh.F0[tid] = F0;
    }
    // ---- support data, one point per thread
    for (int yi = tid; yi < NW * 64; yi += NW * 64) {
      int r = 0, c = 0;
      double nu = 0;
      if (yi < U) {
        split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
        nu = p.uni_nu[ub + yi];
      }
      sh.yrc[yi] = (r << 16) | c;
      sh.nuf[yi] = (float)nu;
    }
    __syncthreads();
    double massmu[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 64; k++) {
      const int qa = block_quadrant(k >> 3, k & 7, p.s);
      if (qa >= 0) massmu[qa] += sh.mu[k];
    }
    const double muJ = (massmu[0] + massmu[1]) + (massmu[2] + massmu[3]);
    const double tol = p.err_tol * muJ;
    const double mux = sh.mu[lane];  // this lane's pixel in the X-update

    float P[8][8];
    int status = 0, loops_all = 0;
    double lam = p.lam;
    constexpr bool quad = QUAD;  // quadratic cost: row and column parts separate
    const int phases = p.safeguard ? 3 : 1;
    bool converged = false, deferred = false;
    double err_last = 0;
    float r_last = 0.f;
    const int xr = g.R0 + xg;  // pixel row of the lane's 8 pixels

    for (int phase = 0; phase < phases; phase++) {
      // the first solve stops at the safeguard trigger, the safeguard's two
      // solves at the loop cap
      const int cap = phase == 0 ? p.cap0 : p.max_iter;
      if (phase == 1) {  // safeguard: 2*eps from the stored potential
        lam = p.lam * 0.5;
        if (tid < 64) sh.F0[tid] = sh.F0orig[tid] * 0.5;
      } else if (phase == 2) {  // back to eps from the 2*eps solution
        lam = p.lam;
        if (tid < 64 && sh.mu[tid] > 0) sh.F0[tid] = (sh.F0[tid] + log((double)uw[tid])) * 2.0;
      }
      float lup = 0.f;  // log2 of the previous iterate's scaling (relative to F0), lane = x
      if (lane == 0) cheb_reset(sh.cheb[wave]);
      __syncthreads();
      // ---- absorb: P = exp(Fmu - lam d2 - m(y)) with Fmu = F0 + log mu
      auto absorb = [&]() {
          if (tid < 64) sh.Fmu[tid] = sh.mu[tid] > 0 ? sh.F0[tid] + log(sh.mu[tid]) : -INFINITY;
          uw[lane] = mux > 0 ? 1.0f : 0.0f;
          __syncthreads();
#pragma unroll
          for (int t = 0; t < 8; t++) {
            const int yi = ybase + t;
            const int rc = sh.yrc[yi];
            const int dr = (rc >> 16) - xr;
            const int dc0 = (rc & 0xffff) - g.C0;
            const double ldr = lam * (double)(dr * dr);
            double mloc = -INFINITY;
#pragma unroll
            for (int j = 0; j < 8; j++) {
              const int dc = dc0 - j;
              const double e = sh.Fmu[xg * 8 + j] - (quad ? ldr + lam * (double)(dc * dc) : lam * cost_q<QUAD>(dr, dc, p.half_p));
              mloc = e > mloc ? e : mloc;
            }
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
              const double v = __shfl_xor(mloc, o, 64);
              mloc = v > mloc ? v : mloc;
            }
            const bool valid = yi < U;
            if (!valid) mloc = 0.0;
#pragma unroll
            for (int j = 0; j < 8; j++) {
              const int dc = dc0 - j;
              const double e = sh.Fmu[xg * 8 + j] - (quad ? ldr + lam * (double)(dc * dc) : lam * cost_q<QUAD>(dr, dc, p.half_p)) - mloc;
              P[j][t] = valid ? fast_exp2((float)(e * kLog2e)) : 0.0f;
            }
            if (xg == 0 && valid) mbuf[yi] = mloc;
          }
        __syncthreads();
      };
      absorb();
      int it = 0;
      converged = false;
      for (;;) {
        it++;
        float (*wred)[64] = sh.wred[it & 1];
        // ---- Y-iteration: S(y) = sum_x P u, w = nu_J / S
        {
          float uu[8], Sp[8];
#pragma unroll
          for (int j = 0; j < 8; j++) uu[j] = uw[xg * 8 + j];
#pragma unroll
          for (int t = 0; t < 8; t++) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < 8; j++) s = fmaf(P[j][t], uu[j], s);
            Sp[t] = s;
          }
          const float s = reduce8_t(Sp, xg);
          const int yi = ybase + xg;
          sh.w[yi] = s > 0.f ? sh.nuf[yi] * __builtin_amdgcn_rcpf(s) : 0.f;
        }
        wave_sync();
        // ---- X-marginal: r(x) = sum_y P w
        {
          float wv[8], rx[8];
#pragma unroll
          for (int t = 0; t < 8; t++) wv[t] = sh.w[ybase + t];
#pragma unroll
          for (int j = 0; j < 8; j++) {
            float s = 0.f;
#pragma unroll
            for (int t = 0; t < 8; t++) s = fmaf(P[j][t], wv[t], s);
            rx[j] = s;
          }
          wred[wave][xg * 8 + yg] = reduce8_j(rx, yg);
        }
        __syncthreads();
        // ---- X-update in every wave: plain u = mu/r, or the accelerated
        // combination of the log-scalings of the current, plain-next and
        // previous iterate; identical in all waves
        float r = 0.f;
#pragma unroll
        for (int w = 0; w < NW; w++) r += wred[w][lane];
        float unew;
        const XUpdate xu = x_update(r, mux, uw[lane], &lup, &unew, tol, it, cap, p.accel,
                                    sh.cheb[wave], lane);
        err_last = xu.err;
        r_last = r;
        if (xu.err <= tol) {
          converged = true;
          break;
        }
        if (!xu.go_on) break;  // cap or non-finite
        uw[lane] = unew;       // own copy: read by this wave only
        if (xu.flag) {
          // exact X-iteration in the log domain:
          //   F0(x) = -LSE_y[G(y) + log nu_J(y) - C(x,y)],  G(y) = -(m(y) + log S(y)),
          // with S(y) = nu_J(y) / w(y) of this loop's Y-iteration
          __syncthreads();  // every wave is done with its partials
          double* dr8 = reinterpret_cast<double*>(rd);  // 256 doubles per wave
#pragma unroll
          for (int j = 0; j < 8; j++) {
            double mm = -INFINITY;
#pragma unroll
            for (int t = 0; t < 8; t++) {
              const int yi = ybase + t;
              const float wy = sh.w[yi], nf = sh.nuf[yi];
              if (yi < U && wy > 0.f && nf > 0.f) {
                const int rc = sh.yrc[yi];
                const int dr = (rc >> 16) - xr, dc = (rc & 0xffff) - (g.C0 + j);
                // G(y) + log nu_J(y) = log w(y) - m(y): the FP32 logarithm of w
                // is enough for the next absorbed potential (the loops go on)
                const double e = (double)(fast_log2(wy) * kLn2f) - mbuf[yi] -
                                 lam * cost_q<QUAD>(dr, dc, p.half_p);
                mm = e > mm ? e : mm;
              }
            }
#pragma unroll
            for (int o = 8; o < 64; o <<= 1) {
              const double v = __shfl_xor(mm, o, 64);
              mm = v > mm ? v : mm;
            }
            if (yg == 0) dr8[xg * 8 + j] = mm;
          }
          __syncthreads();
          if (tid < 64) {
            double mm = -INFINITY;
            for (int w = 0; w < NW; w++) {
              const double v = reinterpret_cast<double*>(sh.red[w])[tid];
              mm = v > mm ? v : mm;
            }
            sh.mx[tid] = mm;
          }
          __syncthreads();
#pragma unroll
          for (int j = 0; j < 8; j++) {
            const double mm = sh.mx[xg * 8 + j];
            double s = 0;
#pragma unroll
            for (int t = 0; t < 8; t++) {
              const int yi = ybase + t;
              const float wy = sh.w[yi], nf = sh.nuf[yi];
              if (yi < U && wy > 0.f && nf > 0.f) {
                const int rc = sh.yrc[yi];
                const int dr = (rc >> 16) - xr, dc = (rc & 0xffff) - (g.C0 + j);
                const double e = (double)(fast_log2(wy) * kLn2f) - mbuf[yi] -
                                 lam * cost_q<QUAD>(dr, dc, p.half_p) - mm;
                s += (double)fast_exp2((float)(e * kLog2e));
              }
            }
#pragma unroll
            for (int o = 8; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
            if (yg == 0) dr8[64 + xg * 8 + j] = s;
          }
          __syncthreads();
          if (tid < 64) {
            float lp = 0.f;
            if (sh.mu[tid] > 0) {
              double s = 0;
              for (int w = 0; w < NW; w++) s += reinterpret_cast<double*>(sh.red[w])[64 + tid];
              const double Fh = -(sh.mx[tid] + log(s));
              // uw was left unchanged by x_update on this path
              const double F = sh.F0[tid] + (double)fast_log2(uw[tid]) * kLn2;
              const double Fp = sh.F0[tid] + (double)lup * kLn2;
              const double Fn = xu.acc ? xu.a * F + xu.b * Fh + xu.d * Fp : Fh;
              sh.F0[tid] = Fn;
              lp = (float)((F - Fn) * kLog2e);
            }
            sh.lupx[tid] = lp;
          }
          __syncthreads();
          lup = sh.lupx[lane];
          absorb();
        }
        if (it == p.newton_after && phase == 0) {
          // hand the cell to the Newton solver with its current potential
          // F0 + log u; the stored potential (alpha) stays for the safeguard
          if (tid < 64)
            p.defer_F[(int64_t)cell * 64 + tid] =
                sh.mu[tid] > 0 ? sh.F0[tid] + log((double)uw[tid]) : 0.0;
          if (tid == 0) {
            const int grp = defer_group(bin);
            const int slot = atomicAdd(&s.defer_count[grp], 1);  // < cap: one per item
            s.defer_list[(int64_t)grp * s.cap + slot] = item;
            p.r_loops[cell] = it;
          }
          deferred = true;
          break;
        }
      }
      __syncthreads();  // every wave has left the loop before the tile or F0 change
      if (deferred) break;
      loops_all += it;
      if (phase == 0) {
        if (converged) break;
        if (phases > 1) status |= 4;
        continue;
      }
      if (phase == 1 && err_last == err_last) continue;  // always return to eps
      break;
    }
    if (deferred) continue;
    if (!converged) status |= (err_last == err_last) ? 1 : 2;

    // ---- final: split of the last Y-iteration by basic cell, cost, objective
    float sl_t, sl_b, sr_t, sr_b, cp;
    {
      float uu[8], v[8];
#pragma unroll
      for (int j = 0; j < 8; j++) uu[j] = uw[xg * 8 + j];
      // left / right basic cells: block columns j < s and j >= s (the block
      // columns from 2s on carry no mass, u = 0 there)
      const int sp = p.s;
#pragma unroll
      for (int t = 0; t < 8; t++) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < 8; j++) s = fmaf(j < sp ? P[j][t] : 0.f, uu[j], s);
        v[t] = s;
      }
      transpose_y(rd, xg, yg, v, &sl_t, &sl_b, sp);
#pragma unroll
      for (int t = 0; t < 8; t++) {
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < 8; j++) s = fmaf(j < sp ? 0.f : P[j][t], uu[j], s);
        v[t] = s;
      }
      transpose_y(rd, xg, yg, v, &sr_t, &sr_b, sp);
#pragma unroll
      for (int t = 0; t < 8; t++) {
        const int yi = ybase + t;
        const int rc = sh.yrc[yi];
        const int dr = (rc >> 16) - xr, dc0 = (rc & 0xffff) - g.C0;
        float s = 0.f;
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int dc = dc0 - j;
          s = fmaf((float)cost_q<QUAD>(dr, dc, p.half_p), P[j][t] * uu[j], s);
        }
        v[t] = s;
      }
      float c1, c2;
      transpose_y(rd, xg, yg, v, &c1, &c2);
      cp = c1 + c2;
    }
    const int yi = ybase + xg;
    const bool own = yi < U;
    int key = 0;
    double vq[4] = {0, 0, 0, 0}, cost_y = 0, obj_y = 0, nuJ = 0;
    if (own) {
      key = p.uni_key[ub + yi];
      nuJ = p.uni_nu[ub + yi];
      const double s0 = sl_t, s1 = sr_t, s2 = sl_b, s3 = sr_b;
      const double S = (s0 + s1) + (s2 + s3);
      vq[0] = nuJ * (s0 / S);
      vq[1] = nuJ * (s1 / S);
      vq[2] = nuJ * (s2 / S);
      vq[3] = nuJ * (s3 / S);
      cost_y = nuJ * ((double)cp / S) * p.hp;
      // nu_J(y) (G(y) + log(nu_J(y)/nu(y))) - nu_J(y),  G(y) = -(m(y) + log S(y))
      const bool key_ok = (unsigned)key < (unsigned)(p.H * p.W);
      if (nuJ > 0 && key_ok) obj_y = nuJ * (-(mbuf[yi] + log(S)) + log(nuJ) - log(p.nu[key])) - nuJ;
    }
    const double cost = block_sum_d(cost_y, sh.out.red);
    double objx = 0;
    if (tid < 64 && sh.mu[tid] > 0) {
      const double F = sh.F0[tid] + log((double)uw[tid]);
      objx = (double)uw[tid] * (double)r_last * F;
    }
    const double obj = block_sum_d(obj_y + objx, sh.out.red);
    if (tid < 4) sh.out.cnt[tid] = 0;
    __syncthreads();
    balance_truncate_write(p, g, obase, U, own, yi, key, vq, massmu, sh.out);
    if (tid == 0) {
#pragma unroll
      for (int a = 0; a < 4; a++)
        if (g.bq[a] >= 0) {
          p.row_off[g.bq[a]] = obase + (int64_t)g.qidx[a] * U;
          p.row_len[g.bq[a]] = (int)min((long long)U, sh.out.cnt[a]);
        }
      p.r_cost[cell] = cost;
      p.r_obj[cell] = p.eps * obj;
      p.r_err[cell] = err_last;
      p.r_loops[cell] = loops_all;
      p.r_status[cell] = status;
      p.r_evals[cell] = (long long)loops_all * p.s * p.s * g.nq * U;
    }
    if (tid < 64 && sh.mu[tid] > 0) {
      const int i = tid >> 3, j = tid & 7;
      p.alpha[(int64_t)(g.R0 + i) * p.W + g.C0 + j] = p.eps * (sh.F0[tid] + log((double)uw[tid]));
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ streamed solver

// Cells whose union exceeds the register capacity (1024 < U <= kStreamMaxU):
// the iteration of the register solver with the absorbed tile kept in a
// per-workgroup global buffer (FP32, written at every absorption, read once
// per loop) and the support processed in slabs of kSlab = 512 points.  Within
// a slab the lane layout is the one of the 8-wave register solver, and the
// Y-iteration and the X-marginal of a slab share one read of its tile:
//   S(y) = sum_x P u  ->  w(y) = nu_J / S  ->  r(x) += sum_y P w.
// The tile of slab s, wave w is stored as 16 float4 per lane, float4 k of
// lane l at ((s*kSW + w)*16 + k)*64 + l, so that every load instruction of a
// wave reads 1 KiB of consecutive memory.  Eight waves leave 256 VGPRs per
// lane for the tile, its scaling vectors and the FP64 bookkeeping.
constexpr int kSW = 8;
constexpr int kSlab = kSW * 64;
static_assert(kStreamMaxU % kSlab == 0, "slabs tile the streamed support");
struct StreamShared {
  double F0[64], Fmu[64], mu[64], F0orig[64], mx[64];
  float u[64], r[64];
  float red[kSW][512];  // per-wave transposition scratch (also FP64 scratch)
  float wred[kSW][64];  // per-wave X partials
  float wl[kSW][64];    // per-wave w of the current slab
  float lup[64];
  ChebState cheb;
  double ca, cb, cd;
  int cacc;
  double err;
  int flag;
  int next;
  CellOutSh out;
};

DEVI float4* tile_at(float* base, int slab, int wave, int k, int lane) {
  return reinterpret_cast<float4*>(base) + ((size_t)((slab * kSW + wave) * 16 + k) * 64 + lane);
}

template <bool QUAD>
__global__ __launch_bounds__(kSlab) void k_solve_stream(const HalfParams* __restrict__ P,
                                                        SweepSched s) {
  __shared__ StreamShared sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int xg = lane & 7, yg = lane >> 3;
  const int yoff = wave * 64 + yg * 8;  // first of the lane's 8 points within a slab
  const int bin = kNBins - 2;
  const int count = s.bin_count[bin];
  float* rd = sh.red[wave];
  float* tileb = s.stream_tile + (size_t)blockIdx.x * kStreamTileFloats;
  float* Sg = s.stream_S + (size_t)blockIdx.x * kStreamMaxU;
  float* nug = s.stream_nu + (size_t)blockIdx.x * kStreamMaxU;
  for (;;) {
    if (tid == 0) sh.next = atomicAdd(&s.queue[bin], 1);
    __syncthreads();
    const int ci = sh.next;
    if (ci >= count) break;
    const int item = __builtin_amdgcn_readfirstlane(s.bin_list[(int64_t)bin * s.cap + ci]);
    const HalfParams& p = P[item >> kItemShift];
    const int cell = item & kItemCellMask;
    const double invW = 1.0 / p.W;
    const CellGeo g = load_geo(p, cell);
    const int U = min(p.cell_U[cell], kStreamMaxU);  // the bin holds U <= kStreamMaxU only
    const int nslab = (U + kSlab - 1) / kSlab;
    const int64_t ub = p.cell_toff[cell];
    const int64_t obase = p.cell_ooff[cell];
    double* mbuf = p.uni_G + ub;  // m(y) of the absorbed tile
    if (tid < 64) {
      const int i = tid >> 3, j = tid & 7;
      const int qa = block_quadrant(i, j, p.s);
      const int bq = qa < 0 ? -1 : qa == 0 ? g.bq[0] : qa == 1 ? g.bq[1] : qa == 2 ? g.bq[2] : g.bq[3];
      const int r = g.R0 + i, c = g.C0 + j;
      double mu = 0, F0 = 0;
      if (bq >= 0) {
        mu = p.mu[(int64_t)r * p.W + c];
        F0 = p.alpha[(int64_t)r * p.W + c] / p.eps;
      }
      sh.mu[tid] = mu;
      sh.F0orig[tid] = F0;
      sh.F0[tid] = F0;
    }
    for (int yi = tid; yi < nslab * kSlab; yi += kSlab) nug[yi] = yi < U ? (float)p.uni_nu[ub + yi] : 0.f;
    __syncthreads();
    double massmu[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 64; k++) {
      const int qa = block_quadrant(k >> 3, k & 7, p.s);
      if (qa >= 0) massmu[qa] += sh.mu[k];
    }
    const double muJ = (massmu[0] + massmu[1]) + (massmu[2] + massmu[3]);
    const double tol = p.err_tol * muJ;

    int status = 0, loops_all = 0;
    double lam = p.lam;
    constexpr bool quad = QUAD;  // quadratic cost: row and column parts separate
    const int phases = p.safeguard ? 3 : 1;
    bool converged = false, deferred = false;
    const int xr = g.R0 + xg;

    for (int phase = 0; phase < phases; phase++) {
      const int cap = phase == 0 ? p.cap0 : p.max_iter;  // safeguard trigger, then loop cap
      if (phase == 1) {
        lam = p.lam * 0.5;
        if (tid < 64) sh.F0[tid] = sh.F0orig[tid] * 0.5;
      } else if (phase == 2) {
        lam = p.lam;
        if (tid < 64 && sh.mu[tid] > 0) sh.F0[tid] = (sh.F0[tid] + log((double)sh.u[tid])) * 2.0;
      }
      if (tid < 64) sh.lup[tid] = 0.f;
      if (tid == 0) cheb_reset(sh.cheb);
      __syncthreads();
      // ---- absorb: tile P = exp(Fmu - lam d2 - m(y)) of every slab to the buffer
      auto absorb = [&]() {
        if (tid < 64) {
          sh.Fmu[tid] = sh.mu[tid] > 0 ? sh.F0[tid] + log(sh.mu[tid]) : -INFINITY;
          sh.u[tid] = sh.mu[tid] > 0 ? 1.0f : 0.0f;
        }
        __syncthreads();
        for (int sl = 0; sl < nslab; sl++)
#pragma unroll
        for (int th = 0; th < 2; th++) {  // four support points at a time
          float P[8][4];
#pragma unroll
          for (int tt = 0; tt < 4; tt++) {
            const int t = th * 4 + tt;
            const int yi = sl * kSlab + yoff + t;
            const bool valid = yi < U;
            int r = 0, c = 0;
            if (valid) split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
            const int dr = r - xr;
            const int dc0 = c - g.C0;
            const double ldr = lam * (double)(dr * dr);
            double mloc = -INFINITY;
#pragma unroll
            for (int j = 0; j < 8; j++) {
              const int dc = dc0 - j;
              const double e = sh.Fmu[xg * 8 + j] - (quad ? ldr + lam * (double)(dc * dc) : lam * cost_q<QUAD>(dr, dc, p.half_p));
              mloc = e > mloc ? e : mloc;
            }
#pragma unroll
            for (int o = 1; o < 8; o <<= 1) {
              const double v = __shfl_xor(mloc, o, 64);
              mloc = v > mloc ? v : mloc;
            }
            if (!valid) mloc = 0.0;
#pragma unroll
            for (int j = 0; j < 8; j++) {
              const int dc = dc0 - j;
              const double e = sh.Fmu[xg * 8 + j] - (quad ? ldr + lam * (double)(dc * dc) : lam * cost_q<QUAD>(dr, dc, p.half_p)) - mloc;
              P[j][tt] = valid ? fast_exp2((float)(e * kLog2e)) : 0.0f;
            }
            if (xg == 0 && valid) mbuf[yi] = mloc;
          }
#pragma unroll
          for (int j = 0; j < 8; j++)
            *tile_at(tileb, sl, wave, 2 * j + th, lane) = make_float4(P[j][0], P[j][1], P[j][2], P[j][3]);
        }
        __syncthreads();
      };
      absorb();
      int it = 0;
      converged = false;
      for (;;) {
        it++;
        // ---- per slab: Y-iteration, w, X-marginal partials
        float uu[8], rx[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          uu[j] = sh.u[xg * 8 + j];
          rx[j] = 0.f;
        }
        for (int sl = 0; sl < nslab; sl++) {
          float P[8][8];
#pragma unroll
          for (int j = 0; j < 8; j++) {
            const float4 a = *tile_at(tileb, sl, wave, 2 * j, lane);
            const float4 b = *tile_at(tileb, sl, wave, 2 * j + 1, lane);
            P[j][0] = a.x; P[j][1] = a.y; P[j][2] = a.z; P[j][3] = a.w;
            P[j][4] = b.x; P[j][5] = b.y; P[j][6] = b.z; P[j][7] = b.w;
          }
          float Sp[8];
#pragma unroll
          for (int t = 0; t < 8; t++) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < 8; j++) s = fmaf(P[j][t], uu[j], s);
            Sp[t] = s;
          }
          const int yi = sl * kSlab + yoff + xg;
          const float S = reduce8_t(Sp, xg);
          const float w = (yi < U && S > 0.f) ? nug[yi] * __builtin_amdgcn_rcpf(S) : 0.f;
          Sg[yi] = S;
          sh.wl[wave][yg * 8 + xg] = w;
          wave_sync();
          float wv[8];
#pragma unroll
          for (int t = 0; t < 8; t++) wv[t] = sh.wl[wave][yg * 8 + t];
#pragma unroll
          for (int j = 0; j < 8; j++)
#pragma unroll
            for (int t = 0; t < 8; t++) rx[j] = fmaf(P[j][t], wv[t], rx[j]);
          wave_sync();
        }
        sh.wred[wave][xg * 8 + yg] = reduce8_j(rx, yg);
        __syncthreads();
        if (wave == 0) {
          float r = 0.f;
#pragma unroll
          for (int w = 0; w < kSW; w++) r += sh.wred[w][lane];
          const double mu = sh.mu[lane];
          const float u = sh.u[lane];
          double e = mu > 0 ? fabs((double)u * (double)r - mu) : 0.0;
          e = wave_sum(e);
          sh.r[lane] = r;
          const bool go_on = !(e <= tol) && it < cap && (e == e);
          if (lane == 0) {
            double a0 = 0, b0 = 1, d0 = 0;
            const bool acc0 = go_on && p.accel && cheb_next(sh.cheb, it, e, &a0, &b0, &d0);
            sh.cacc = acc0;
            sh.ca = a0;
            sh.cb = b0;
            sh.cd = d0;
          }
          wave_sync();
          const bool acc = sh.cacc;
          const double a = sh.ca, b = sh.cb, d = sh.cd;
          const float un = mu > 0 ? (float)(mu / (double)r) : 0.f;
          const float lu = mu > 0 ? fast_log2(u) : 0.f;
          float unew = un;
          if (acc && mu > 0) {
            const float ln = fast_log2(un);
            unew = fast_exp2((float)(a * lu + b * ln + d * sh.lup[lane]));
          }
          const bool bad = mu > 0 && !(unew > 9.357623e-14f && unew < 1.0686475e13f &&
                                       un > 0.f && un < 3.0e38f);
          const unsigned long long anyb = __ballot(bad);
          if (go_on && anyb == 0ull) {
            sh.u[lane] = unew;
            sh.lup[lane] = lu;
          }
          if (lane == 0) {
            sh.err = e;
            sh.flag = go_on && anyb != 0ull;
          }
        }
        __syncthreads();
        const double err = sh.err;
        if (err <= tol) {
          converged = true;
          break;
        }
        if (!(err == err) || it >= cap) break;
        if (sh.flag) {
          // exact X-iteration in the log domain over all slabs:
          //   F0(x) = -LSE_y[G(y) + log nu_J(y) - C(x,y)],  G(y) = -(m(y) + log S(y))
          double* dr8 = reinterpret_cast<double*>(rd);
          double mm[8];
#pragma unroll
          for (int j = 0; j < 8; j++) mm[j] = -INFINITY;
          for (int sl = 0; sl < nslab; sl++)
#pragma unroll
            for (int t = 0; t < 8; t++) {
              const int yi = sl * kSlab + yoff + t;
              if (yi < U) {
                const float S = Sg[yi], nf = nug[yi];
                if (S > 0.f && nf > 0.f) {
                  int r, c;
                  split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
                  const int dr = r - xr;
                  const double gl = -(mbuf[yi] + log((double)S)) + log((double)nf) -
                                    (quad ? lam * (double)(dr * dr) : 0.0);
#pragma unroll
                  for (int j = 0; j < 8; j++) {
                    const int dc = c - (g.C0 + j);
                    const double e = gl - (quad ? lam * (double)(dc * dc)
                                                : lam * cost_q<QUAD>(dr, dc, p.half_p));
                    mm[j] = e > mm[j] ? e : mm[j];
                  }
                }
              }
            }
#pragma unroll
          for (int j = 0; j < 8; j++) {
#pragma unroll
            for (int o = 8; o < 64; o <<= 1) {
              const double v = __shfl_xor(mm[j], o, 64);
              mm[j] = v > mm[j] ? v : mm[j];
            }
          }
          wave_sync();
          if (yg == 0)
#pragma unroll
            for (int j = 0; j < 8; j++) dr8[xg * 8 + j] = mm[j];
          __syncthreads();
          if (tid < 64) {
            double m = -INFINITY;
            for (int w = 0; w < kSW; w++) {
              const double v = reinterpret_cast<double*>(sh.red[w])[tid];
              m = v > m ? v : m;
            }
            sh.mx[tid] = m;
          }
          __syncthreads();
          double sj[8];
#pragma unroll
          for (int j = 0; j < 8; j++) sj[j] = 0.0;
          for (int sl = 0; sl < nslab; sl++)
#pragma unroll
            for (int t = 0; t < 8; t++) {
              const int yi = sl * kSlab + yoff + t;
              if (yi < U) {
                const float S = Sg[yi], nf = nug[yi];
                if (S > 0.f && nf > 0.f) {
                  int r, c;
                  split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
                  const int dr = r - xr;
                  const double gl = -(mbuf[yi] + log((double)S)) + log((double)nf) -
                                    (quad ? lam * (double)(dr * dr) : 0.0);
#pragma unroll
                  for (int j = 0; j < 8; j++) {
                    const int dc = c - (g.C0 + j);
                    const double e = gl - (quad ? lam * (double)(dc * dc)
                                                : lam * cost_q<QUAD>(dr, dc, p.half_p)) -
                                     sh.mx[xg * 8 + j];
                    sj[j] += (double)fast_exp2((float)(e * kLog2e));
                  }
                }
              }
            }
#pragma unroll
          for (int j = 0; j < 8; j++) {
#pragma unroll
            for (int o = 8; o < 64; o <<= 1) sj[j] += __shfl_xor(sj[j], o, 64);
          }
          if (yg == 0)
#pragma unroll
            for (int j = 0; j < 8; j++) dr8[64 + xg * 8 + j] = sj[j];
          __syncthreads();
          if (tid < 64 && sh.mu[tid] > 0) {
            double s = 0;
            for (int w = 0; w < kSW; w++) s += reinterpret_cast<double*>(sh.red[w])[64 + tid];
            const double Fh = -(sh.mx[tid] + log(s));
            const double F = sh.F0[tid] + (double)fast_log2(sh.u[tid]) * kLn2;
            const double Fp = sh.F0[tid] + (double)sh.lup[tid] * kLn2;
            const double Fn = sh.cacc ? sh.ca * F + sh.cb * Fh + sh.cd * Fp : Fh;
            sh.F0[tid] = Fn;
            sh.lup[tid] = (float)((F - Fn) * kLog2e);
          }
          __syncthreads();
          absorb();
        }
        if (it == p.newton_after && phase == 0) {
          if (tid < 64)
            p.defer_F[(int64_t)cell * 64 + tid] =
                sh.mu[tid] > 0 ? sh.F0[tid] + log((double)sh.u[tid]) : 0.0;
          if (tid == 0) {
            const int grp = defer_group(bin);
            const int slot = atomicAdd(&s.defer_count[grp], 1);  // < cap: one per item
            s.defer_list[(int64_t)grp * s.cap + slot] = item;
            p.r_loops[cell] = it;
          }
          deferred = true;
          break;
        }
      }
      if (deferred) break;
      loops_all += it;
      if (phase == 0) {
        if (converged) break;
        if (phases > 1) status |= 4;
        continue;
      }
      if (phase == 1 && sh.err == sh.err) continue;  // always return to eps
      break;
    }
    if (deferred) {
      __syncthreads();
      continue;
    }
    if (!converged) status |= (sh.err == sh.err) ? 1 : 2;

    // ---- final: split of the last Y-iteration by basic cell, cost, objective,
    // stashed per support point in the output region, then balanced and compacted
    if (tid < 4) sh.out.cnt[tid] = 0;
    double cost_acc = 0, obj_acc = 0;
    {
      float uu[8];
#pragma unroll
      for (int j = 0; j < 8; j++) uu[j] = sh.u[xg * 8 + j];
      for (int sl = 0; sl < nslab; sl++) {
        float P[8][8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const float4 a = *tile_at(tileb, sl, wave, 2 * j, lane);
          const float4 b = *tile_at(tileb, sl, wave, 2 * j + 1, lane);
          P[j][0] = a.x; P[j][1] = a.y; P[j][2] = a.z; P[j][3] = a.w;
          P[j][4] = b.x; P[j][5] = b.y; P[j][6] = b.z; P[j][7] = b.w;
        }
        float sl_t, sl_b, sr_t, sr_b, c1, c2, v[8];
        const int sp = p.s;  // left / right basic cells: block columns j < s, j >= s
#pragma unroll
        for (int t = 0; t < 8; t++) {
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < 8; j++) s = fmaf(j < sp ? P[j][t] : 0.f, uu[j], s);
          v[t] = s;
        }
        transpose_y(rd, xg, yg, v, &sl_t, &sl_b, sp);
#pragma unroll
        for (int t = 0; t < 8; t++) {
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < 8; j++) s = fmaf(j < sp ? 0.f : P[j][t], uu[j], s);
          v[t] = s;
        }
        transpose_y(rd, xg, yg, v, &sr_t, &sr_b, sp);
#pragma unroll
        for (int t = 0; t < 8; t++) {
          const int yi = sl * kSlab + yoff + t;
          int r = 0, c = 0;
          if (yi < U) split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
          const int dr = r - xr, dc0 = c - g.C0;
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < 8; j++) {
            const int dc = dc0 - j;
            s = fmaf((float)cost_q<QUAD>(dr, dc, p.half_p), P[j][t] * uu[j], s);
          }
          v[t] = s;
        }
        transpose_y(rd, xg, yg, v, &c1, &c2);
        const int yi = sl * kSlab + yoff + xg;
        if (yi < U) {
          const int key = p.uni_key[ub + yi];
          const double nuJ = p.uni_nu[ub + yi];
          const double s0 = sl_t, s1 = sr_t, s2 = sl_b, s3 = sr_b;
          const double S = (s0 + s1) + (s2 + s3);
          const double vq[4] = {nuJ * (s0 / S), nuJ * (s1 / S), nuJ * (s2 / S), nuJ * (s3 / S)};
          cost_acc += nuJ * ((double)(c1 + c2) / S) * p.hp;
          const bool key_ok = (unsigned)key < (unsigned)(p.H * p.W);
          if (nuJ > 0 && key_ok)
            obj_acc += nuJ * (-(mbuf[yi] + log(S)) + log(nuJ) - log(p.nu[key])) - nuJ;
#pragma unroll
          for (int a = 0; a < 4; a++)
            if (g.bq[a] >= 0) {
              const int64_t at = obase + (int64_t)g.qidx[a] * U + yi;
              p.ent_val[at] = vq[a];
              p.ent_col[at] = key;
            }
        }
        wave_sync();
      }
    }
    __syncthreads();
    balance_compact_chunked(p, g, obase, U, massmu, sh.out);
    const double cost = block_sum_d(cost_acc, sh.out.red);
    double objx = 0;
    if (tid < 64 && sh.mu[tid] > 0) {
      const double F = sh.F0[tid] + log((double)sh.u[tid]);
      objx = (double)sh.u[tid] * (double)sh.r[tid] * F;
    }
    const double obj = block_sum_d(obj_acc + objx, sh.out.red);
    if (tid == 0) {
#pragma unroll
      for (int a = 0; a < 4; a++)
        if (g.bq[a] >= 0) {
          p.row_off[g.bq[a]] = obase + (int64_t)g.qidx[a] * U;
          p.row_len[g.bq[a]] = (int)min((long long)U, sh.out.cnt[a]);
        }
      p.r_cost[cell] = cost;
      p.r_obj[cell] = p.eps * obj;
      p.r_err[cell] = sh.err;
      p.r_loops[cell] = loops_all;
      p.r_status[cell] = status;
      p.r_evals[cell] = (long long)loops_all * p.s * p.s * g.nq * U;
    }
    if (tid < 64 && sh.mu[tid] > 0) {
      const int i = tid >> 3, j = tid & 7;
      p.alpha[(int64_t)(g.R0 + i) * p.W + g.C0 + j] = p.eps * (sh.F0[tid] + log((double)sh.u[tid]));
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ big-cell solver

// Cells whose union exceeds the register capacity, and cells handed over by
// the register solver for Newton steps.  The Sinkhorn iteration is evaluated
// in the log domain on every pass (FP64 exponents, FP32 exponentials, FP64
// sums), potentials G(y) kept in the union scratch.
//
// Newton fallback (same rule as the oracle): after `newton_after` loops the
// cell problem is maximised over the X potential alone (the semi-dual
//   Phi(F) = sum_x mu F - sum_y nu_J(y) log sum_x exp(F - C) mu,
// Y potential eliminated by the exact Y-iteration).  Gradient mu - r, minus
// the Hessian is the Laplacian of W(x,x') = sum_y nu_J p_x(y) p_x'(y) with
// p_x(y) the conditional plan.  Each iteration: one Y-iteration (the loop and
// its stopping test), W in FP64, the grounded Laplacian system solved by
// subtraction-free (GTH) elimination, the step capped to max|d| <= 8, then a
// backtracking Armijo search on the increase of Phi evaluated as
//   <g, a> - sum_y nu_J log(sum_x p_x (e^(a - c_y))),  c_y = sum_x p_x a,
// (two non-negative sums) and, if no trial passes, a plain X-iteration.
// Waves per workgroup: 8 for the log-domain solver of the largest bin, 16 for
// the Newton launches (one tail cell then holds a compute unit alone, and
// twice the waves hide more of the FP64 latency).
constexpr int kBigWaves = 8;
constexpr int kNewtonWaves = 16;
constexpr int kNewtonMaxSteps = 100;
constexpr double kNewtonStepCap = 8.0;
constexpr int kNewtonTrials = 10;
constexpr double kNewtonArmijo = 1e-4;

template <int NW>
struct BigShared {
  static constexpr int kNChunk = NW * 4;  // support points per Newton chunk (16 threads each)
  double F[64], Fmu[64], mu[64], Fh[64], F0orig[64], Fp[64];
  double r[64], b[64], dl[64], piv[64];
  ChebState cheb;
  double ca, cb, cd;
  int cacc;
  int xr[64], xc[64];
  union {
    struct {
      double pm[NW][64], ps[NW][64];
    } lse;                       // Sinkhorn X-marginal partials
    double q[64][kNChunk + 1];   // Newton: p_x(y) sqrt(nu_J(y)) of one chunk of support points
    double racc[NW][64];         // Newton: X-marginal partials per wave
  } u;
  double Wm[64][65];             // Newton: weights W(x,x'), eliminated in place
  double err, slope;
  int last;                // last active pixel (ground of the Laplacian system)
  int nact;                // active pixels (mu > 0)
  int next;
  CellOutSh out;
};

// e^b - 1 - b >= 0 without cancellation, in FP32 (relative error ~1e-7):
// Taylor series through b^9 for |b| < 1/2, else exp - 1 - b
DEVI float phi1f(float b) {
  if (fabsf(b) < 0.5f) {
    float t = 1.f / 362880.f;
    t = fmaf(t, b, 1.f / 40320.f);
    t = fmaf(t, b, 1.f / 5040.f);
    t = fmaf(t, b, 1.f / 720.f);
    t = fmaf(t, b, 1.f / 120.f);
    t = fmaf(t, b, 1.f / 24.f);
    t = fmaf(t, b, 1.f / 6.f);
    t = fmaf(t, b, 0.5f);
    return b * b * t;
  }
  return (fast_exp2(b * (float)kLog2e) - 1.f) - b;
}

typedef double doublex4 __attribute__((ext_vector_type(4)));

// Sum / max over the 16 lanes of a DPP row (quad swaps and row rotations, so
// every lane ends with the result).
DEVI double row16_sum(double v) {
  v += dpp_d<0xb1>(v);
  v += dpp_d<0x4e>(v);
  v += dpp_d<0x124>(v);
  v += dpp_d<0x128>(v);
  return v;
}
DEVI double row16_max(double v) {
  v = fmax(v, dpp_d<0xb1>(v));
  v = fmax(v, dpp_d<0x4e>(v));
  v = fmax(v, dpp_d<0x124>(v));
  v = fmax(v, dpp_d<0x128>(v));
  return v;
}

// e^x in FP64 or through the FP32 exponential (x <= 0 in every use)
DEVI double ex(double x, bool fp64) {
  return fp64 ? exp(x) : (double)fast_exp2((float)(x * kLog2e));
}

// e^b - 1 - b in FP64 (series for small |b|, no cancellation)
DEVI double phi1d(double b) {
  if (fabs(b) < 1e-3) return b * b * (0.5 + b * (1.0 / 6 + b * (1.0 / 24 + b / 120)));
  return expm1(b) - b;
}

// Conditional plan of support point yi for the 4 pixels xs + 16k of this
// thread (16 threads per support point, lanes xs = tid & 15 of a 16-lane
// group): pk[k] = p_x(y), returns m + log s (= -G(y)).  prec 0: FP32
// exponentials (plain iterations); 1: FP64 exponentials (the Newton system);
// 2: FP64 exponentials and logarithm (FP64 instantiation).  s lies in
// [1, 64] (the largest term is e^0), so the FP32 logarithm is accurate to
// ~1e-7 absolute.
template <bool QUAD, class SH>
DEVI double cond_plan(const SH& sh, int r, int c, int xs, double lam, double half_p,
                      double pk[4], int prec) {
  double e[4];
  double m = -INFINITY;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int x = xs + 16 * k;
    const int dr = r - sh.xr[x], dc = c - sh.xc[x];
    e[k] = sh.Fmu[x] - lam * cost_q<QUAD>(dr, dc, half_p);
    m = e[k] > m ? e[k] : m;
  }
  m = row16_max(m);
  double v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    // the plans of far-apart pixels underflow FP32, and the Newton system
    // needs exactly those weak couplings
    v[k] = e[k] == -INFINITY ? 0.0
           : prec > 0       ? exp(e[k] - m)
                            : (double)fast_exp2((float)((e[k] - m) * kLog2e));
    s += v[k];
  }
  s = row16_sum(s);
  const double inv = 1.0 / s;
#pragma unroll
  for (int k = 0; k < 4; k++) pk[k] = v[k] * inv;
  return m + (prec == 2 ? log(s) : (double)fast_log2((float)s) * kLn2);
}

template <int NW, bool QUAD>
__global__ __launch_bounds__(NW * 64) void k_solve_big(const HalfParams* __restrict__ P,
                                                       SweepSched s, int mode) {
  constexpr int kBigThreads = NW * 64, kNChunk = BigShared<NW>::kNChunk;
  constexpr int kTiles = 16 / NW;  // 16x16 tiles of W per wave
  __shared__ BigShared<NW> sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int yl = tid >> 4, xs = tid & 15;  // Newton layout: kNChunk support points x 16 threads
  const bool deferred = mode >= 1;
  const int grp = mode - 1;  // Newton group of the handed-over cells
  const int count = deferred ? s.defer_count[grp] : s.bin_count[kNBins - 1];
  for (;;) {
    if (tid == 0) sh.next = atomicAdd(&s.queue[deferred ? kNBins + grp : kNBins - 1], 1);
    __syncthreads();
    const int ci = sh.next;
    if (ci >= count) break;
    const int item = __builtin_amdgcn_readfirstlane(
        deferred ? s.defer_list[(int64_t)grp * s.cap + ci]
                 : s.bin_list[(int64_t)(kNBins - 1) * s.cap + ci]);
    const HalfParams& p = P[item >> kItemShift];
    const int cell = item & kItemCellMask;
    const double invW = 1.0 / p.W;
    const bool fp64 = p.fp64 != 0;
    const CellGeo g = load_geo(p, cell);
    const int U = p.cell_U[cell];
    const int64_t ub = p.cell_toff[cell];
    const int64_t obase = p.cell_ooff[cell];
    if (tid < 64) {
      const int i = tid >> 3, j = tid & 7;
      const int qa = block_quadrant(i, j, p.s);
      const int r = g.R0 + i, c = g.C0 + j;
      double mu = 0, F = 0, F0 = 0;
      const int bq = qa < 0 ? -1 : qa == 0 ? g.bq[0] : qa == 1 ? g.bq[1] : qa == 2 ? g.bq[2] : g.bq[3];
      if (bq >= 0) {
        mu = p.mu[(int64_t)r * p.W + c];
        F0 = p.alpha[(int64_t)r * p.W + c] / p.eps;
        F = deferred ? p.defer_F[(int64_t)cell * 64 + tid] : F0;
      }
      sh.mu[tid] = mu;
      sh.F[tid] = F;
      sh.F0orig[tid] = F0;
      sh.xr[tid] = r;
      sh.xc[tid] = c;
      const unsigned long long act = __ballot(mu > 0);
      if (tid == 0) {
        sh.last = act ? 63 - __builtin_clzll(act) : -1;
        sh.nact = __builtin_popcountll(act);
      }
    }
    __syncthreads();
    double massmu[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < 64; k++) {
      const int qa = block_quadrant(k >> 3, k & 7, p.s);
      if (qa >= 0) massmu[qa] += sh.mu[k];
    }
    const double tol = p.err_tol * (massmu[0] + massmu[1] + massmu[2] + massmu[3]);
    const int n_act = sh.nact;
    double* G = p.uni_G + ub;
    int status = 0, loops_all = 0;
    // work of a handed-over cell in this launch: loops before the hand-over,
    // line-search passes and W formations (Newton steps)
    const int pre_loops = deferred ? p.r_loops[cell] : 0;
    long long n_trials = 0, n_wbuild = 0;
    bool converged = false;
    double lam = p.lam;
    constexpr bool quad = QUAD;  // quadratic cost: row and column parts separate
    const int phases = p.safeguard ? 3 : 1;
    for (int phase = 0; phase < phases; phase++) {
      const int cap = phase == 0 ? p.cap0 : p.max_iter;  // safeguard trigger, then loop cap
      if (phase == 1) {
        lam = p.lam * 0.5;
        if (tid < 64) sh.F[tid] = sh.F0orig[tid] * 0.5;
      } else if (phase == 2) {
        lam = p.lam;
        if (tid < 64) sh.F[tid] *= 2.0;
      }
      __syncthreads();
      if (tid < 64) {
        sh.Fmu[tid] = sh.mu[tid] > 0 ? sh.F[tid] + log(sh.mu[tid]) : -INFINITY;
        sh.Fp[tid] = sh.F[tid];
      }
      if (tid == 0) cheb_reset(sh.cheb);
      __syncthreads();
      bool newton = deferred && phase == 0;
      int it = newton ? p.r_loops[cell] : 0;
      while (!newton) {
        it++;
        // Y-iteration
        for (int yi = tid; yi < U; yi += kBigThreads) {
          int r, c;
          split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
          double m = -INFINITY;
          for (int k = 0; k < 64; k++) {
            const int dr = r - sh.xr[k], dc = c - sh.xc[k];
            const double e = sh.Fmu[k] - lam * cost_q<QUAD>(dr, dc, p.half_p);
            m = e > m ? e : m;
          }
          double s = 0;
          for (int k = 0; k < 64; k++) {
            const int dr = r - sh.xr[k], dc = c - sh.xc[k];
            const double e = sh.Fmu[k] - lam * cost_q<QUAD>(dr, dc, p.half_p) - m;
            s += ex(e, fp64);
          }
          const double nu = p.uni_nu[ub + yi];
          G[yi] = -(m + log(s)) + (nu > 0 ? log(nu) : -INFINITY);  // G(y) + log nu_J(y)
        }
        __syncthreads();
        // X-marginal: Fh(x) = -LSE_y[G(y) + log nu_J(y) - C(x,y)], online per thread
        {
          const int x = lane;
          double m = -INFINITY, s = 0;
          for (int yi = wave; yi < U; yi += NW) {
            int r, c;
            split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
            const int dr = r - sh.xr[x], dc = c - sh.xc[x];
            const double e = G[yi] - lam * cost_q<QUAD>(dr, dc, p.half_p);
            if (e == -INFINITY) continue;
            if (e > m) {
              s = s * ex(m - e, fp64) + 1.0;
              m = e;
            } else {
              s += ex(e - m, fp64);
            }
          }
          sh.u.lse.pm[wave][x] = m;
          sh.u.lse.ps[wave][x] = s;
        }
        __syncthreads();
        if (wave == 0) {
          double m = -INFINITY;
          for (int w = 0; w < NW; w++) m = sh.u.lse.pm[w][lane] > m ? sh.u.lse.pm[w][lane] : m;
          double s = 0;
          for (int w = 0; w < NW; w++)
            if (sh.u.lse.ps[w][lane] > 0) s += sh.u.lse.ps[w][lane] * exp(sh.u.lse.pm[w][lane] - m);
          const double Fh = -(m + log(s));
          sh.Fh[lane] = Fh;
          const double mu = sh.mu[lane];
          double e = mu > 0 ? mu * fabs(exp(sh.F[lane] - Fh) - 1.0) : 0.0;
          e = wave_sum(e);
          if (lane == 0) {
            double a0 = 0, b0 = 1, d0 = 0;
            const bool go_on = !(e <= tol) && it < cap && (e == e);
            sh.cacc = go_on && p.accel && cheb_next(sh.cheb, it, e, &a0, &b0, &d0);
            sh.ca = a0;
            sh.cb = b0;
            sh.cd = d0;
            sh.err = e;
          }
        }
        __syncthreads();
        const double err = sh.err;
        if (err <= tol) {
          converged = true;
          break;
        }
        if (!(err == err) || it >= cap) break;
        if (tid < 64 && sh.mu[tid] > 0) {
          const double F = sh.F[tid];
          const double Fn = sh.cacc ? sh.ca * F + sh.cb * sh.Fh[tid] + sh.cd * sh.Fp[tid] : sh.Fh[tid];
          sh.Fp[tid] = F;
          sh.F[tid] = Fn;
          sh.Fmu[tid] = Fn + log(sh.mu[tid]);
        }
        __syncthreads();
        if (it == p.newton_after) newton = true;
      }
      if (newton) {
        status |= 16;
        int nst = 0;
        for (;;) {
          it++;
          const bool build_w = nst < kNewtonMaxSteps && n_act > 1;
          // ---- Y-iteration with conditional plans, X-marginal r, weights W
          double racc[4] = {0, 0, 0, 0};
          // W = Q Q^T by FP64 matrix cores, 16x16 tiles.  The couplings of far-apart
          // pixels are tiny and the Newton step follows the smallest
          // eigenvalues of the Laplacian, so W is formed and eliminated in FP64.
          // wave w owns the tiles t = kTiles w + j: rows 16 (t >> 2), columns 16 (t & 3)
          doublex4 wacc[kTiles] = {};
          const int wr = 16 * ((kTiles * wave) >> 2) + (lane & 15);  // row of Q for operand A
          const int wc = 16 * ((kTiles * wave) & 3) + (lane & 15);   // row of Q for operand B
          const int wk = lane >> 4;                                  // k within a step of 4
          for (int y0 = 0; y0 < U; y0 += kNChunk) {
            const int yi = y0 + yl;
            double pk[4] = {0, 0, 0, 0};
            double sq = 0;
            if (yi < U) {  // uniform within each 16-lane group
              int r, c;
              split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
              const double lse = cond_plan<QUAD>(sh, r, c, xs, lam, p.half_p, pk, fp64 ? 2 : build_w ? 1 : 0);
              const double nu = p.uni_nu[ub + yi];
#pragma unroll
              for (int k = 0; k < 4; k++) racc[k] += nu * pk[k];
              if (xs == 0) G[yi] = -lse + (nu > 0 ? log(nu) : -INFINITY);
              sq = sqrt(nu);
            }
            if (build_w) {
#pragma unroll
              for (int k = 0; k < 4; k++) sh.u.q[xs + 16 * k][yl] = pk[k] * sq;
              __syncthreads();
#pragma unroll
              for (int k0 = 0; k0 < kNChunk; k0 += 4) {
                const double a = sh.u.q[wr][k0 + wk];
#pragma unroll
                for (int j = 0; j < kTiles; j++)
                  wacc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, sh.u.q[wc + 16 * j][k0 + wk],
                                                                 wacc[j], 0, 0, 0);
              }
              __syncthreads();
            }
          }
#pragma unroll
          for (int k = 0; k < 4; k++) {
            racc[k] += __shfl_xor(racc[k], 16, 64);
            racc[k] += __shfl_xor(racc[k], 32, 64);
          }
          if (lane < 16)
#pragma unroll
            for (int k = 0; k < 4; k++) sh.u.racc[wave][lane + 16 * k] = racc[k];
          if (build_w)
#pragma unroll
            for (int v = 0; v < 4; v++) {  // D(i,j): i = 4v + lane/16, j = lane%16
              const int i = wr - (lane & 15) + 4 * v + (lane >> 4);
#pragma unroll
              for (int j = 0; j < kTiles; j++) sh.Wm[i][wc + 16 * j] = wacc[j][v];
            }
          __syncthreads();
          if (wave == 0) {
            double r = 0;
            for (int w = 0; w < NW; w++) r += sh.u.racc[w][lane];
            const double mu = sh.mu[lane];
            if (!(mu > 0)) r = 0;
            sh.r[lane] = r;
            const double e = wave_sum_dpp(mu > 0 ? fabs(r - mu) : 0.0);
            if (lane == 0) sh.err = e;
          }
          __syncthreads();
          const double err = sh.err;
          if (err <= tol) {
            converged = true;
            break;
          }
          if (!(err == err) || it >= cap) break;
          bool step = false;
          double t = 1.0;
          if (build_w) {
            nst++;
            n_wbuild++;
            // right side g - r sum(g)/sum(r), g = mu - r
            if (wave == 0) {
              const double mu = sh.mu[lane], r = sh.r[lane];
              const double gx = mu > 0 ? mu - r : 0.0;
              const double sg = wave_sum_dpp(gx), sr = wave_sum_dpp(r);
              sh.b[lane] = gx - r * (sg / sr);
            }
            __syncthreads();
            // subtraction-free (GTH) elimination of the Laplacian of W in LDS,
            // grounded at the last active pixel: the pivot of row k is the sum
            // of its remaining weights (every wave reduces it itself), then the
            // trailing weights take W(i,k) W(k,j) / d_k, one row per wave
            const int last = sh.last;
            for (int k = 0; k < last; k++) {
              const double dk = wave_sum_dpp(lane > k ? sh.Wm[k][lane] : 0.0);
              if (tid == 0) sh.piv[k] = dk;
              if (dk > 0) {
                const double inv = 1.0 / dk;
                if (wave == 0 && lane > k) sh.b[lane] += sh.Wm[lane][k] * inv * sh.b[k];
                for (int i = k + 1 + wave; i < 64; i += NW) {
                  const double c = sh.Wm[i][k] * inv;
                  if (lane > k && lane != i && c != 0) sh.Wm[i][lane] += c * sh.Wm[k][lane];
                }
              }
              __syncthreads();
            }
            if (wave == 0) {
              // back substitution from the ground down: d_k = (b_k + sum_{j>k} W(k,j) d_j) / d_k
              double dl = 0;  // lane k: d_k
              for (int k = last - 1; k >= 0; k--) {
                const double sk = wave_sum_dpp(lane > k ? sh.Wm[k][lane] * dl : 0.0);
                const double pv = sh.piv[k];
                const double dk = pv > 0 ? (sh.b[k] + sk) / pv : 0.0;
                if (lane == k) dl = dk;
              }
              const double mu = sh.mu[lane];
              const double gx = mu > 0 ? mu - sh.r[lane] : 0.0;
              double dx = dl;
              const double dm = wave_max(fabs(dx));
              if (dm > kNewtonStepCap) dx *= kNewtonStepCap / dm;
              sh.dl[lane] = dx;
              const double sl = wave_sum_dpp(gx * dx);
              if (lane == 0) sh.slope = sl;
            }
            __syncthreads();
            const double slope = sh.slope;
            if (slope > 0) {
              for (int trial = 0; trial < kNewtonTrials; trial++) {
                n_trials++;
                double loc = 0;
                for (int y0 = 0; y0 < U; y0 += kNChunk) {
                  const int yi = y0 + yl;
                  if (yi < U) {
                    int r, c;
                    split_key(p.uni_key[ub + yi], p.W, invW, &r, &c);
                    double pk[4];
                    cond_plan<QUAD>(sh, r, c, xs, lam, p.half_p, pk, fp64 ? 2 : 1);
                    double a[4], cy = 0;
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                      a[k] = t * sh.dl[xs + 16 * k];
                      cy += pk[k] * a[k];
                    }
                    cy = row16_sum(cy);
                    double sp = 0;
#pragma unroll
                    for (int k = 0; k < 4; k++)
                      sp += pk[k] > 0 ? pk[k] * (fp64 ? phi1d(a[k] - cy)
                                                      : (double)phi1f((float)(a[k] - cy)))
                                      : 0.0;
                    sp = row16_sum(sp);
                    if (xs == 0) loc -= p.uni_nu[ub + yi] * log1p(sp);
                  }
                }
                if (tid < 64) {
                  const double mu = sh.mu[tid];
                  loc += mu > 0 ? (mu - sh.r[tid]) * t * sh.dl[tid] : 0.0;
                }
                const double inc = block_sum_d(loc, sh.out.red);
                if (inc >= kNewtonArmijo * t * slope) {
                  step = true;
                  break;
                }
                t *= 0.5;
              }
            }
          }
          if (tid < 64 && sh.mu[tid] > 0) {
            const double F = step ? sh.F[tid] + t * sh.dl[tid]
                                  : sh.F[tid] + log(sh.mu[tid]) - log(sh.r[tid]);
            sh.F[tid] = F;
            sh.Fmu[tid] = F + log(sh.mu[tid]);
          }
          __syncthreads();
        }
        // X-marginal of the last Y-iteration as mu exp(F - Fh) (final pass)
        if (tid < 64)
          sh.Fh[tid] = sh.mu[tid] > 0 ? sh.F[tid] - log(sh.r[tid] / sh.mu[tid]) : 0.0;
        __syncthreads();
      }
      loops_all += it;
      if (phase == 0) {
        if (converged) break;
        if (phases > 1) status |= 4;
        continue;
      }
      if (phase == 1 && sh.err == sh.err) continue;  // always return to eps
      break;
    }
    if (!converged) status |= (sh.err == sh.err) ? 1 : 2;
    // final split / cost / objective, chunked over the support
    if (tid < 4) sh.out.cnt[tid] = 0;
    __syncthreads();
    double cost_acc = 0, obj_acc = 0;
    for (int y0 = 0; y0 < U; y0 += kBigThreads) {
      const int yi = y0 + tid;
      const bool own = yi < U;
      double vq[4] = {0, 0, 0, 0};
      int key = 0;
      if (own) {
        key = p.uni_key[ub + yi];
        int r, c;
        split_key(key, p.W, invW, &r, &c);
        const double gl = G[yi];
        double sq[4] = {0, 0, 0, 0}, cs = 0;
        // plan column: pi(x,y) = exp(F(x) + log mu(x) + G(y) + log nu_J(y) - C(x,y))
        double m = -INFINITY;
        for (int k = 0; k < 64; k++) {
          const int dr = r - sh.xr[k], dc = c - sh.xc[k];
          const double e = sh.Fmu[k] - lam * cost_q<QUAD>(dr, dc, p.half_p);
          m = e > m ? e : m;
        }
        for (int k = 0; k < 64; k++) {
          const int dr = r - sh.xr[k], dc = c - sh.xc[k];
          const double cu = cost_q<QUAD>(dr, dc, p.half_p);
          const double e = sh.Fmu[k] - lam * cu - m;
          const double v = ex(e, fp64);
          const int qa = block_quadrant(k >> 3, k & 7, p.s);
          sq[0] += qa == 0 ? v : 0.0;
          sq[1] += qa == 1 ? v : 0.0;
          sq[2] += qa == 2 ? v : 0.0;
          sq[3] += qa == 3 ? v : 0.0;
          cs += v * cu;
        }
        const double nuJ = p.uni_nu[ub + yi];
        const double S = sq[0] + sq[1] + sq[2] + sq[3];
        _Pragma("unroll") for (int a = 0; a < 4; a++) vq[a] = nuJ * (sq[a] / S);
        cost_acc += nuJ * (cs / S) * p.hp;
        const double Gy = gl - (nuJ > 0 ? log(nuJ) : 0.0);
        const bool key_ok = (unsigned)key < (unsigned)(p.H * p.W);
        obj_acc += (nuJ > 0 && key_ok) ? nuJ * (Gy + log(nuJ) - log(p.nu[key])) - nuJ : 0.0;
      }
      // chunk-wise norms are accumulated by the balancing helper only for one
      // chunk; large cells therefore balance in a second pass below
      if (own) {
        // stash the unbalanced split in the output region (segment per quadrant)
        _Pragma("unroll") for (int a = 0; a < 4; a++)
          if (g.bq[a] >= 0) {
            const int64_t at = obase + (int64_t)g.qidx[a] * U + yi;
            p.ent_val[at] = vq[a];
            p.ent_col[at] = key;
          }
      }
    }
    __syncthreads();
    balance_compact_chunked(p, g, obase, U, massmu, sh.out);
    const double cost = block_sum_d(cost_acc, sh.out.red);
    double objx = 0;
    if (tid < 64 && sh.mu[tid] > 0) {
      // X-marginal of the final plan is mu(x) exp(F - Fh)
      objx = sh.mu[tid] * exp(sh.F[tid] - sh.Fh[tid]) * sh.F[tid];
    }
    const double obj = block_sum_d(obj_acc + objx, sh.out.red);
    if (tid == 0) {
      _Pragma("unroll") for (int a = 0; a < 4; a++)
        if (g.bq[a] >= 0) {
          p.row_off[g.bq[a]] = obase + (int64_t)g.qidx[a] * U;
          p.row_len[g.bq[a]] = (int)min((long long)U, sh.out.cnt[a]);
        }
      p.r_cost[cell] = cost;
      p.r_obj[cell] = p.eps * obj;
      p.r_err[cell] = sh.err;
      p.r_loops[cell] = loops_all;
      p.r_status[cell] = status;
      int nx = 0;
      _Pragma("unroll") for (int a = 0; a < 4; a++) nx += g.bq[a] >= 0 ? p.s * p.s : 0;
      if (deferred) {
        // the solver that handed the cell over keeps its own loops; this
        // launch counts its passes over the support (loops and line-search
        // trials) and the FP64 matrix-core flops of W = Q Q^T (64x64xU)
        p.r_evals[cell] = (long long)pre_loops * nx * U;
        p.r_nev[cell] = (long long)(loops_all - pre_loops + n_trials) * nx * U;
        p.r_nmf[cell] = n_wbuild * 2LL * 64 * 64 * U;
      } else {
        p.r_evals[cell] = (long long)loops_all * nx * U;
      }
    }
    if (tid < 64 && sh.mu[tid] > 0)
      p.alpha[sh.xr[tid] * p.W + sh.xc[tid]] = p.eps * sh.F[tid] * (lam / p.lam);
    __syncthreads();
  }
}

// ------------------------------------------------------------ warm-start features

// Features of one composite cell problem for the warm-start network, 256
// threads per cell.  Positions are in pixels of the level; the cell's integer
// shift d_J = round(mean_nu(y) - mean_mu(x)) moves the nu window onto the
// cell, and the X potentials are written for the problem with cost
// |x - (y - d_J)|^2: F~ = F + 2 lam (x - x_c).d_J, centred over the pixels of
// positive mass (x_c the block centre, lam = h^2/eps), so that they carry no
// bulk linear trend.  The network predicts the change of F~ that the cell
// solve will make to the potential it starts from (zero output = the plain
// warm start).
//   [0, 64)     64 mu(x) / |mu_J| on the 8x8 block (0 where a quadrant is absent)
//   [64, 640)   256 nu_J(y) / |nu_J| on the 24x24 window whose rows start at
//               R0 - 8 + d_r and columns at C0 - 8 + d_c
//   640         log lam,  641  nu_J mass outside the window / |nu_J|,
//   642, 643    d_J / 8
//   [644, 708)  F~ of the starting potential / (kWarmScale lam)
//   rest 0
// Leaves the features in sh.f, d_J in *dr, *dc and the centred F~ of the
// potential `alpha` (units of eps) of this thread's pixel (threads < 64) in
// *ft (0 for pixels without mass).
struct FeatShared {
  float f[kFeatIn];
  double red[8];
};

DEVI void cell_features(const HalfParams& p, const CellGeo& g, int U, int64_t ub,
                        const double* alpha, FeatShared& sh, int* dr_out, int* dc_out,
                        double* ft_out) {
  const int tid = threadIdx.x;
  const double invW = 1.0 / p.W;
  for (int k = tid; k < kFeatIn; k += blockDim.x) sh.f[k] = 0.f;
  // mu block: mass and mass-weighted position
  double mu = 0, mr = 0, mc = 0;
  int64_t px = 0;
  if (tid < 64) {
    const int i = tid >> 3, j = tid & 7;
    const int qa = block_quadrant(i, j, p.s);
    const int bq = qa < 0 ? -1 : qa == 0 ? g.bq[0] : qa == 1 ? g.bq[1] : qa == 2 ? g.bq[2] : g.bq[3];
    px = (int64_t)(g.R0 + i) * p.W + g.C0 + j;
    if (bq >= 0) {
      mu = p.mu[px];
      mr = mu * i;
      mc = mu * j;
    }
  }
  const double mm = block_sum_d(mu, sh.red);
  mr = block_sum_d(mr, sh.red);
  mc = block_sum_d(mc, sh.red);
  // nu_J: mass and mass-weighted position (relative to the block origin)
  double nm = 0, nr = 0, nc = 0;
  for (int y = tid; y < U; y += blockDim.x) {
    int r, c;
    split_key(p.uni_key[ub + y], p.W, invW, &r, &c);
    const double v = p.uni_nu[ub + y];
    nm += v;
    nr += v * (r - g.R0);
    nc += v * (c - g.C0);
  }
  nm = block_sum_d(nm, sh.red);
  nr = block_sum_d(nr, sh.red);
  nc = block_sum_d(nc, sh.red);
  const int dr = (int)rint(nm > 0 && mm > 0 ? nr / nm - mr / mm : 0.0);
  const int dc = (int)rint(nm > 0 && mm > 0 ? nc / nm - mc / mm : 0.0);
  // starting potential, shift-compensated and centred
  double ft = 0, act = 0;
  if (tid < 64 && mu > 0) {
    const int i = tid >> 3, j = tid & 7;
    ft = alpha[px] / p.eps + 2.0 * p.lam * ((i - 3.5) * dr + (j - 3.5) * dc);
    act = 1;
  }
  const double fsum = block_sum_d(ft, sh.red), na = block_sum_d(act, sh.red);
  if (act > 0) ft -= fsum / na;
  if (tid < 64 && mm > 0) {
    sh.f[tid] = (float)(64.0 * mu / mm);
    sh.f[644 + tid] = (float)(ft / (kWarmScale * p.lam));
  }
  double out = 0;
  for (int y = tid; y < U; y += blockDim.x) {
    int r, c;
    split_key(p.uni_key[ub + y], p.W, invW, &r, &c);
    const double v = nm > 0 ? p.uni_nu[ub + y] / nm : 0.0;
    const int wr = r - (g.R0 - 8 + dr), wc = c - (g.C0 - 8 + dc);
    if (wr >= 0 && wr < 24 && wc >= 0 && wc < 24)
      sh.f[64 + wr * 24 + wc] = (float)(256.0 * v);  // keys are unique: one point per pixel
    else
      out += v;
  }
  out = block_sum_d(out, sh.red);
  if (tid == 0) {
    sh.f[640] = (float)log(p.lam);
    sh.f[641] = (float)out;
    sh.f[642] = dr * 0.125f;
    sh.f[643] = dc * 0.125f;
  }
  __syncthreads();
  *dr_out = dr;
  *dc_out = dc;
  *ft_out = act > 0 ? ft : 0.0;
}

DEVI unsigned short bf16_bits_rn(float f) {
  const unsigned u = __float_as_uint(f);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// Inference input of a sweep: one BF16 row per cell (zero for cells whose
// union exceeds kWarmMaxU), from the potentials the sweep starts from.
__global__ __launch_bounds__(256) void k_warm_features(HalfParams p, unsigned short* X) {
  __shared__ FeatShared sh;
  for (int cell = blockIdx.x; cell < p.n_cells; cell += gridDim.x) {
    const int U = p.cell_U[cell];
    if (U > kWarmMaxU) {
      for (int k = threadIdx.x; k < kFeatIn; k += blockDim.x) X[(size_t)cell * kFeatIn + k] = 0;
      continue;  // uniform
    }
    const CellGeo g = load_geo(p, cell);
    int dr, dc;
    double ft;
    cell_features(p, g, U, p.cell_toff[cell], p.alpha, sh, &dr, &dc, &ft);
    for (int k = threadIdx.x; k < kFeatIn; k += blockDim.x)
      X[(size_t)cell * kFeatIn + k] = bf16_bits_rn(sh.f[k]);
    __syncthreads();
  }
}

// Warm start of eligible cells: the network output Y is the change of the
// centred F~ in units of kWarmScale lam, so F0 = alpha / eps + kWarmScale lam Y
// (the shift's linear part cancels), written over alpha for the cell's pixels
// of positive mass -- for cells whose predicted change has an RMS of at least
// min_rms (in output units) only; the others keep the plain start.
__global__ __launch_bounds__(64) void k_warm_apply(HalfParams p, const float* Y, float min_rms,
                                                   int* n_applied) {
  const int cell = blockIdx.x;
  if (cell >= p.n_cells || p.cell_U[cell] > kWarmMaxU) return;  // uniform
  const CellGeo g = load_geo(p, cell);
  const int i = threadIdx.x >> 3, j = threadIdx.x & 7;
  const int qa = block_quadrant(i, j, p.s);
  const int bq = qa < 0 ? -1 : qa == 0 ? g.bq[0] : qa == 1 ? g.bq[1] : qa == 2 ? g.bq[2] : g.bq[3];
  const int64_t px = (int64_t)(g.R0 + i) * p.W + g.C0 + j;
  const bool act = bq >= 0 && p.mu[px] > 0;
  const double y = act ? (double)Y[(size_t)cell * 64 + threadIdx.x] : 0.0;
  const double ss = wave_sum_dpp(y * y), na = wave_sum_dpp(act ? 1.0 : 0.0);
  if (!(na > 0) || ss < (double)min_rms * min_rms * na) return;  // uniform
  if (act) p.alpha[px] += p.eps * kWarmScale * p.lam * y;
  if (threadIdx.x == 0) atomicAdd(n_applied, 1);
}

// Training samples of the last sweep: the features of each converged cell
// with U <= kWarmMaxU built from the potentials the sweep started from
// (alpha_prev), the change of the centred F~ that the solve made (alpha after
// the sweep minus alpha_prev, in units of kWarmScale lam) and the mask of
// pixels with positive mass; rows appended at an atomic counter.
__global__ __launch_bounds__(256) void k_collect(HalfParams p, const double* alpha_prev, float* X,
                                                 float* T, float* M, int* ids, int cap,
                                                 int* count) {
  __shared__ FeatShared sh;
  __shared__ int slot;
  for (int cell = blockIdx.x; cell < p.n_cells; cell += gridDim.x) {
    const int U = p.cell_U[cell];
    if (U > kWarmMaxU || p.r_status[cell] != 0) continue;  // uniform
    const CellGeo g = load_geo(p, cell);
    int dr, dc;
    double f0, f1;
    cell_features(p, g, U, p.cell_toff[cell], p.alpha, sh, &dr, &dc, &f1);  // converged F~
    __syncthreads();
    cell_features(p, g, U, p.cell_toff[cell], alpha_prev, sh, &dr, &dc, &f0);  // start
    if (threadIdx.x == 0) slot = atomicAdd(count, 1);
    __syncthreads();
    const int s = slot;
    if (s < cap) {
      if (ids && threadIdx.x == 0) ids[s] = cell;
      for (int k = threadIdx.x; k < kFeatIn; k += blockDim.x) X[(size_t)s * kFeatIn + k] = sh.f[k];
      if (threadIdx.x < 64) {
        const bool a = sh.f[threadIdx.x] > 0.f;  // mu > 0
        T[(size_t)s * 64 + threadIdx.x] = a ? (float)((f1 - f0) / (kWarmScale * p.lam)) : 0.f;
        M[(size_t)s * 64 + threadIdx.x] = a ? 1.f : 0.f;
      }
    }
    __syncthreads();
  }
}

void launch_warm_features(const HalfParams& p, unsigned short* X, hipStream_t st) {
  hipLaunchKernelGGL(k_warm_features, dim3(p.n_cells < 4096 ? p.n_cells : 4096), dim3(256), 0, st,
                     p, X);
}
void launch_warm_apply(const HalfParams& p, const float* Y, float min_rms, int* n_applied,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_warm_apply, dim3(p.n_cells), dim3(64), 0, st, p, Y, min_rms, n_applied);
}
void launch_collect(const HalfParams& p, const double* alpha_prev, float* X, float* T, float* M,
                    int* ids, int cap, int* count, hipStream_t st) {
  hipLaunchKernelGGL(k_collect, dim3(p.n_cells < 4096 ? p.n_cells : 4096), dim3(256), 0, st, p,
                     alpha_prev, X, T, M, ids, cap, count);
}

// ------------------------------------------------------------ stats

__global__ __launch_bounds__(1024) void k_stats(const HalfParams* __restrict__ P,
                                                IterStatsDev* out) {
  const HalfParams& p = P[blockIdx.x];
  out += blockIdx.x;
  __shared__ double shd[16];
  __shared__ long long shl[16];
  double c = 0, o = 0, e = 0;
  long long lt = 0, ev = 0, nnz = 0, nev = 0, nmf = 0;
  int lmax = 0, nf = 0, ns = 0, nn = 0;
  for (int i = threadIdx.x; i < p.n_cells; i += 1024) {
    c += p.r_cost[i];
    o += p.r_obj[i];
    e += p.r_err[i];
    lt += p.r_loops[i];
    ev += p.r_evals[i];
    // cells handed to a Newton launch (Newton flag, not the log-domain bin,
    // whose solver switches in place): the work of that launch
    if ((p.r_status[i] & 16) && cell_bin(p, p.cell_U[i]) != kNBins - 1) {
      nev += p.r_nev[i];
      nmf += p.r_nmf[i];
    }
    lmax = max(lmax, p.r_loops[i]);
    nf += (p.r_status[i] & 3) != 0;
    ns += (p.r_status[i] & 4) != 0;
    nn += (p.r_status[i] & 16) != 0;
  }
  for (int b = threadIdx.x; b < p.n_basic; b += 1024) nnz += p.row_len[b];
  long long eb[kNBins];
  int cb[kNBins];
#pragma unroll
  for (int k = 0; k < kNBins; k++) {
    eb[k] = 0;
    cb[k] = 0;
  }
  for (int i = threadIdx.x; i < p.n_cells; i += 1024) {
    const int b = cell_bin(p, p.cell_U[i]);
#pragma unroll
    for (int k = 0; k < kNBins; k++) {
      eb[k] += b == k ? p.r_evals[i] : 0;
      cb[k] += b == k;
    }
  }
  c = block_sum_d(c, shd);
  o = block_sum_d(o, shd);
  e = block_sum_d(e, shd);
  long long tot;
  block_excl_scan(lt, shl, &tot);
  lt = tot;
  block_excl_scan(ev, shl, &tot);
  ev = tot;
  block_excl_scan(nnz, shl, &tot);
  nnz = tot;
  block_excl_scan(nev, shl, &tot);
  nev = tot;
  block_excl_scan(nmf, shl, &tot);
  nmf = tot;
  block_excl_scan((long long)nf, shl, &tot);
  nf = (int)tot;
  block_excl_scan((long long)ns, shl, &tot);
  ns = (int)tot;
  block_excl_scan((long long)nn, shl, &tot);
  nn = (int)tot;
#pragma unroll
  for (int k = 0; k < kNBins; k++) {
    long long t2;
    block_excl_scan(eb[k], shl, &t2);
    eb[k] = t2;
    block_excl_scan((long long)cb[k], shl, &t2);
    cb[k] = (int)t2;
  }
  int lm = wave_max(lmax);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) shl[threadIdx.x >> 6] = lm;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long m = 0;
    for (int w = 0; w < 16; w++) m = max(m, shl[w]);
    out->cost = c;
    out->obj = o;
    out->err = e;
    out->loops_total = lt;
    out->evals = ev;
    out->newton_evals = nev;
    out->newton_mfma = nmf;
    out->nnz = nnz;
    out->out_entries = p.misc[1];
    out->bad_rows = p.misc[2];
    out->loops_max = (int)m;
    out->n_failed = nf;
    out->n_safeguard = ns;
    out->n_newton = nn;
    out->n_cells = p.n_cells;
    for (int k = 0; k < kNBins; k++) {
      out->evals_bin[k] = eb[k];
      out->cells_bin[k] = cb[k];
    }
  }
}

// ------------------------------------------------------------ launchers

void launch_sweep_prep(const HalfParams* P, const SweepSched& s, const SweepStreams& ss,
                       const SweepGrid& gr, hipEvent_t* ev) {
  auto pre = [&](int k, hipStream_t st) {
    if (ev) hipEventRecord(ev[2 * k], st);
  };
  auto post = [&](int k, hipStream_t st) {
    if (ev) hipEventRecord(ev[2 * k + 1], st);
  };
  hipStream_t st = ss.main;
  pre(0, st);
  hipLaunchKernelGGL(k_scan_T, dim3(s.n_prob), dim3(1024), 0, st, P);
  post(0, st);
  pre(1, st);
  hipLaunchKernelGGL(k_union, dim3(gr.other, s.n_prob), dim3(kUnionThreads), 0, st, P);
  post(1, st);
  pre(2, st);
  hipLaunchKernelGGL(k_scan_out, dim3(s.n_prob), dim3(1024), 0, st, P);
  hipLaunchKernelGGL(k_sched, dim3(s.n_prob), dim3(256), 0, st, P, s);
  post(2, st);
}

template <bool QUAD>
static void launch_solvers(const HalfParams* P, const SweepSched& s, const SweepStreams& ss,
                           const SweepGrid& gr, hipEvent_t* ev) {
  auto pre = [&](int k, hipStream_t st) {
    if (ev) hipEventRecord(ev[2 * k], st);
  };
  auto post = [&](int k, hipStream_t st) {
    if (ev) hipEventRecord(ev[2 * k + 1], st);
  };
  hipStream_t st = ss.main;
  // fork: the heaviest bins on their own streams, the light ones on main; each
  // stream ends with the Newton launch for the cells its solvers handed over
  // (events kNKernels + i of ev for the three auxiliary ones)
  hipEventRecord(ss.fork, st);
  for (int i = 0; i < 3; i++) hipStreamWaitEvent(ss.aux[i], ss.fork, 0);
  const int gs = gr.bin[5] < s.stream_wgs ? gr.bin[5] : s.stream_wgs;  // one tile buffer per workgroup
  pre(8, ss.aux[0]);
  if (gs > 0) hipLaunchKernelGGL(k_solve_stream<QUAD>, dim3(gs), dim3(kSlab), 0, ss.aux[0], P, s);
  post(8, ss.aux[0]);
  pre(9, ss.aux[0]);
  hipLaunchKernelGGL((k_solve_big<kBigWaves, QUAD>), dim3(gr.bin[6]), dim3(kBigWaves * 64), 0, ss.aux[0], P, s, 0);
  post(9, ss.aux[0]);
  pre(kNKernels + 0, ss.aux[0]);
  hipLaunchKernelGGL((k_solve_big<kNewtonWaves, QUAD>), dim3(gr.newton), dim3(kNewtonWaves * 64), 0, ss.aux[0], P, s, 1 + 3);
  post(kNKernels + 0, ss.aux[0]);
  // the small-cell bins go first on their streams: launched behind the
  // persistent workgroups of the large bins they would wait for free compute
  // units until those drain
  pre(4, ss.aux[1]);
  hipLaunchKernelGGL((k_solve_reg<2, QUAD>), dim3(gr.bin[1]), dim3(128), 0, ss.aux[1], P, s, 1);
  post(4, ss.aux[1]);
  pre(7, ss.aux[1]);
  hipLaunchKernelGGL((k_solve_reg<16, QUAD>), dim3(gr.bin[4]), dim3(1024), 0, ss.aux[1], P, s, 4);
  post(7, ss.aux[1]);
  pre(kNKernels + 1, ss.aux[1]);
  hipLaunchKernelGGL((k_solve_big<kNewtonWaves, QUAD>), dim3(gr.newton), dim3(kNewtonWaves * 64), 0, ss.aux[1], P, s, 1 + 2);
  post(kNKernels + 1, ss.aux[1]);
  pre(3, ss.aux[2]);
  hipLaunchKernelGGL((k_solve_reg<1, QUAD>), dim3(gr.bin[0]), dim3(64), 0, ss.aux[2], P, s, 0);
  post(3, ss.aux[2]);
  pre(6, ss.aux[2]);
  hipLaunchKernelGGL((k_solve_reg<8, QUAD>), dim3(gr.bin[3]), dim3(512), 0, ss.aux[2], P, s, 3);
  post(6, ss.aux[2]);
  pre(kNKernels + 2, ss.aux[2]);
  hipLaunchKernelGGL((k_solve_big<kNewtonWaves, QUAD>), dim3(gr.newton), dim3(kNewtonWaves * 64), 0, ss.aux[2], P, s, 1 + 1);
  post(kNKernels + 2, ss.aux[2]);
  pre(5, st);
  hipLaunchKernelGGL((k_solve_reg<4, QUAD>), dim3(gr.bin[2]), dim3(256), 0, st, P, s, 2);
  post(5, st);
  pre(10, st);
  hipLaunchKernelGGL((k_solve_big<kNewtonWaves, QUAD>), dim3(gr.newton), dim3(kNewtonWaves * 64), 0, st, P, s, 1 + 0);
  post(10, st);
  // join
  for (int i = 0; i < 3; i++) {
    hipEventRecord(ss.join[i], ss.aux[i]);
    hipStreamWaitEvent(st, ss.join[i], 0);
  }
}

void launch_sweep_solve(const HalfParams* P, const SweepSched& s, const SweepStreams& ss,
                        const SweepGrid& gr, hipEvent_t* ev) {
  if (s.quad)
    launch_solvers<true>(P, s, ss, gr, ev);
  else
    launch_solvers<false>(P, s, ss, gr, ev);
}

size_t sweep_max_static_lds() {
  const void* ks[] = {(const void*)k_union,
                      (const void*)k_solve_reg<1, true>, (const void*)k_solve_reg<2, true>,
                      (const void*)k_solve_reg<4, true>, (const void*)k_solve_reg<8, true>,
                      (const void*)k_solve_reg<16, true>, (const void*)k_solve_big<kBigWaves, true>,
                      (const void*)k_solve_big<kNewtonWaves, true>,
                      (const void*)k_solve_reg<1, false>, (const void*)k_solve_reg<2, false>,
                      (const void*)k_solve_reg<4, false>, (const void*)k_solve_reg<8, false>,
                      (const void*)k_solve_reg<16, false>,
                      (const void*)k_solve_big<kBigWaves, false>,
                      (const void*)k_solve_big<kNewtonWaves, false>};
  size_t mx = 0;
  for (const void* k : ks) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, k) == hipSuccess && a.sharedSizeBytes > mx) mx = a.sharedSizeBytes;
  }
  return mx;
}

void launch_stats(const HalfParams* P, int n_prob, IterStatsDev* out, hipStream_t st,
                  hipEvent_t* ev2) {
  if (ev2) hipEventRecord(ev2[0], st);
  hipLaunchKernelGGL(k_stats, dim3(n_prob), dim3(1024), 0, st, P, out);
  if (ev2) hipEventRecord(ev2[1], st);
}

// ------------------------------------------------------------ setup kernels

__global__ __launch_bounds__(1024) void k_validate(const double* mu, const double* nu, int S, int H,
                                                   int W, double* out4) {
  __shared__ double sh[16];
  double sm = 0, sn = 0, bad = 0;
  for (long long i = threadIdx.x; i < (long long)H * W; i += 1024) {
    double a = mu[i], b = nu[i];
    if (!(a >= 0) || !(b >= 0) || !isfinite(a) || !isfinite(b)) bad += 1;
    sm += a;
    sn += b;
  }
  // smallest basic-cell mass of mu
  const int bh = H / S, bw = W / S;
  double mn = INFINITY;
  for (int b = threadIdx.x; b < bh * bw; b += 1024) {
    int br = b / bw, bc = b % bw;
    double m = 0;
    for (int i = 0; i < S; i++)
      for (int j = 0; j < S; j++) m += mu[(long long)(br * S + i) * W + bc * S + j];
    mn = m < mn ? m : mn;
  }
  sm = block_sum_d(sm, sh);
  sn = block_sum_d(sn, sh);
  bad = block_sum_d(bad, sh);
  double mw = wave_min(mn);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mw;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = INFINITY;
    for (int w = 0; w < 16; w++) m = sh[w] < m ? sh[w] : m;
    out4[0] = sm;
    out4[1] = sn;
    out4[2] = bad;
    out4[3] = m;
  }
}

void launch_validate(const double* mu, const double* nu, int s, int H, int W, double* out4,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_validate, dim3(1), dim3(1024), 0, st, mu, nu, s, H, W, out4);
}

__global__ void k_pyramid(const double* fine, double* coarse, int Hc, int Wc) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)Hc * Wc) return;
  int r = (int)(i / Wc), c = (int)(i % Wc);
  const int Wf = 2 * Wc;
  coarse[i] = (fine[(2LL * r) * Wf + 2 * c] + fine[(2LL * r) * Wf + 2 * c + 1]) +
              (fine[(2LL * r + 1) * Wf + 2 * c] + fine[(2LL * r + 1) * Wf + 2 * c + 1]);
}

void launch_pyramid(const double* fine, double* coarse, int Hc, int Wc, hipStream_t st) {
  long long n = (long long)Hc * Wc;
  hipLaunchKernelGGL(k_pyramid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fine, coarse,
                     Hc, Wc);
}

__global__ void k_product_init(const int* ypos, int nzy, const double* nu, const double* bmass,
                               int n_basic, int* col, double* val, int64_t* row_off,
                               int* row_len) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n_basic) {
    row_off[i] = i * (long long)nzy;
    row_len[i] = nzy;
  }
  if (i >= (long long)n_basic * nzy) return;
  int b = (int)(i / nzy), k = (int)(i % nzy);
  col[i] = ypos[k];
  val[i] = bmass[b] * nu[ypos[k]];
}

void launch_product_init(const int* ypos, int nzy, const double* nu, const double* bmass,
                         int n_basic, int* col, double* val, int64_t* row_off, int* row_len,
                         hipStream_t st) {
  long long n = (long long)n_basic * nzy;
  if (n < n_basic) n = n_basic;
  hipLaunchKernelGGL(k_product_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ypos,
                     nzy, nu, bmass, n_basic, col, val, row_off, row_len);
}

// ------------------------------------------------------------ diagnostics

__global__ void k_diag_scatter(const int64_t* row_off, const int* row_len, const int* col,
                               const double* val, int n_basic, double* acc) {
  int b = blockIdx.x;
  if (b >= n_basic) return;
  const int64_t o = row_off[b];
  for (int k = threadIdx.x; k < row_len[b]; k += blockDim.x) atomicAdd(&acc[col[o + k]], val[o + k]);
}

// Partial sums of the diagnostics, one slot per block (grid-stride over
// pixels and basic cells), then a fixed-order sum of the slots.
__global__ __launch_bounds__(256) void k_diag_partial(const int64_t* row_off, const int* row_len,
                                                      const double* val, const double* mu,
                                                      const double* nu, const double* acc, int S,
                                                      int H, int W, int bw, int n_basic,
                                                      double* part) {
  __shared__ double sh[16];
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double ey = 0, dm = 0, nnz = 0;
  for (long long i = t0; i < (long long)H * W; i += stride) ey += fabs(acc[i] - nu[i]);
  for (long long b = t0; b < n_basic; b += stride) {
    double m = 0, mm = 0;
    const int64_t o = row_off[b];
    for (int k = 0; k < row_len[b]; k++) m += val[o + k];
    const int br = (int)(b / bw), bc = (int)(b % bw);
    for (int i = 0; i < S; i++)
      for (int j = 0; j < S; j++) mm += mu[(long long)(br * S + i) * W + bc * S + j];
    dm += fabs(m - mm);
    nnz += row_len[b];
  }
  ey = block_sum_d(ey, sh);
  dm = block_sum_d(dm, sh);
  nnz = block_sum_d(nnz, sh);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = ey;
    part[3 * blockIdx.x + 1] = dm;
    part[3 * blockIdx.x + 2] = nnz;
  }
}

__global__ void k_diag_final(const double* part, int n, double* out3) {
  if (threadIdx.x < 3) {
    double s = 0;
    for (int k = 0; k < n; k++) s += part[3 * k + threadIdx.x];
    out3[threadIdx.x] = s;
  }
}

__global__ void k_zero_d(double* p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

void launch_diag(const int64_t* row_off, const int* row_len, const int* col, const double* val,
                 const double* mu, const double* nu, int s, int H, int W, int bw,
                 int n_basic, double* scratch_px, double* out3, hipStream_t st) {
  // the accumulator is cleared by a kernel (no memset node if a caller captures the launches)
  const long long npx = (long long)H * W;
  const unsigned zb = (unsigned)std::min<long long>((npx + 255) / 256, 4096);
  hipLaunchKernelGGL(k_zero_d, dim3(zb > 0 ? zb : 1), dim3(256), 0, st, scratch_px, npx);
  hipLaunchKernelGGL(k_diag_scatter, dim3(n_basic), dim3(64), 0, st, row_off, row_len, col, val,
                     n_basic, scratch_px);
  // the slots live behind the H*W accumulator (scratch_px holds H*W + 3*kDiagBlocks)
  double* part = scratch_px + (size_t)H * W;
  hipLaunchKernelGGL(k_diag_partial, dim3(kDiagBlocks), dim3(256), 0, st, row_off, row_len, val,
                     mu, nu, scratch_px, s, H, W, bw, n_basic, part);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, part, kDiagBlocks, out3);
}

// ------------------------------------------------------------ export

__global__ __launch_bounds__(1024) void k_scan_rows(const int* row_len, int n, int64_t* row_ptr) {
  __shared__ long long sh[16];
  long long carry = 0;
  for (int base = 0; base < n; base += 1024) {
    int i = base + threadIdx.x;
    long long v = i < n ? row_len[i] : 0;
    long long tot;
    long long ex = block_excl_scan(v, sh, &tot);
    if (i < n) row_ptr[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) row_ptr[n] = carry;
}

void launch_scan_rows(const int* row_len, int n, int64_t* row_ptr, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(1024), 0, st, row_len, n, row_ptr);
}

__global__ void k_export(const int64_t* row_off, const int* row_len, const int* col,
                         const double* val, int n_basic, const int64_t* row_ptr, int* col_out,
                         double* val_out) {
  int b = blockIdx.x;
  if (b >= n_basic) return;
  const int64_t o = row_off[b], d = row_ptr[b];
  for (int k = threadIdx.x; k < row_len[b]; k += blockDim.x) {
    col_out[d + k] = col[o + k];
    val_out[d + k] = val[o + k];
  }
}

void launch_export(const int64_t* row_off, const int* row_len, const int* col, const double* val,
                   int n_basic, int64_t* row_ptr_dev, int* col_out, double* val_out,
                   hipStream_t st) {
  launch_scan_rows(row_len, n_basic, row_ptr_dev, st);
  hipLaunchKernelGGL(k_export, dim3(n_basic), dim3(64), 0, st, row_off, row_len, col, val,
                     n_basic, row_ptr_dev, col_out, val_out);
}

// ------------------------------------------------------------ refinement

// Fine basic marginals by eq. (FineBasicMarginals):
//   nu_i(y) = nu(y) * nuhat_{Pa(i)}(pa(y)) / nuhat(pa(y)) * mu(X_i) / muhat(Xhat_{Pa(i)}).
// Every coarse support point has four children; the fine row is written in
// increasing linear index: for each run of parent points on one coarse row,
// first the children on the upper fine row, then those on the lower one.
__global__ __launch_bounds__(64) void k_refine_fill(RefineParams r) {
  const int b = blockIdx.x;
  if (b >= r.n_basic_f) return;
  const int br = b / r.bwf, bc = b % r.bwf;
  const int P = (br >> 1) * r.bwc + (bc >> 1);
  const int pr = P / r.bwc, pc = P % r.bwc;
  double mi = 0, mP = 0;
  for (int i = 0; i < r.s; i++)
    for (int j = 0; j < r.s; j++) {
      mi += r.mu_f[(long long)(br * r.s + i) * r.Wf + bc * r.s + j];
      mP += r.mu_c[(long long)(pr * r.s + i) * r.Wc + pc * r.s + j];
    }
  const double ratio_mu = mi / mP;
  const int64_t po = r.row_off_c[P];
  const int L = r.row_len_c[P];
  const int64_t fo = r.row_off_f[b];
  const int* key = r.col_c + po;
  for (int k = threadIdx.x; k < L; k += 64) {
    const int y = key[k];
    const int yr = y / r.Wc, yc = y - (y / r.Wc) * r.Wc;
    // run of parent points on coarse row yr: [s, e)
    int lo = 0, hi = L;
    const int k0 = yr * r.Wc;
    while (lo < hi) {
      int m = (lo + hi) >> 1;
      if (key[m] < k0) lo = m + 1; else hi = m;
    }
    const int s = lo;
    lo = s;
    hi = L;
    const int k1 = k0 + r.Wc;
    while (lo < hi) {
      int m = (lo + hi) >> 1;
      if (key[m] < k1) lo = m + 1; else hi = m;
    }
    const int e = lo;
    const double f = r.val_c[po + k] / r.nu_c[y] * ratio_mu;
    for (int u = 0; u < 2; u++)
      for (int v = 0; v < 2; v++) {
        const int64_t idx = 4LL * s + (int64_t)u * 2 * (e - s) + 2LL * (k - s) + v;
        const int yf = (2 * yr + u) * r.Wf + 2 * yc + v;
        r.col_f[fo + idx] = yf;
        r.val_f[fo + idx] = r.nu_f[yf] * f;
      }
  }
}

__global__ void k_refine_rows_len(RefineParams r) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= r.n_basic_f) return;
  const int br = b / r.bwf, bc = b % r.bwf;
  const int P = (br >> 1) * r.bwc + (bc >> 1);
  r.row_len_f[b] = 4 * r.row_len_c[P];
}

void launch_refine_rows(const RefineParams& r, hipStream_t st) {
  hipLaunchKernelGGL(k_refine_rows_len, dim3((r.n_basic_f + 255) / 256), dim3(256), 0, st, r);
  launch_scan_rows(r.row_len_f, r.n_basic_f, r.row_off_f, st);
  hipLaunchKernelGGL(k_refine_fill, dim3(r.n_basic_f), dim3(64), 0, st, r);
}

__global__ void k_glue_ratios(RefineParams r, double* out) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  const int bh = r.Hc / r.s;
  if (b >= bh * r.bwc) return;
  const int br = b / r.bwc, bc = b % r.bwc;
  for (int sgn = 0; sgn < 2; sgn++) {
    const double sg = sgn == 0 ? 1.0 : -1.0;
    double m = -INFINITY;
    for (int i = 0; i < r.s; i++)
      for (int j = 0; j < r.s; j++) {
        long long px = (long long)(br * r.s + i) * r.Wc + bc * r.s + j;
        if (r.mu_c[px] > 0) {
          double v = sg * (r.alpha_a_c[px] - r.alpha_b_c[px]) / r.eps;
          m = v > m ? v : m;
        }
      }
    double acc = 0, tot = 0;
    for (int i = 0; i < r.s; i++)
      for (int j = 0; j < r.s; j++) {
        long long px = (long long)(br * r.s + i) * r.Wc + bc * r.s + j;
        if (r.mu_c[px] > 0) {
          acc += r.mu_c[px] * exp(sg * (r.alpha_a_c[px] - r.alpha_b_c[px]) / r.eps - m);
          tot += r.mu_c[px];
        }
      }
    out[2 * b + sgn] = m + log(acc / tot);
  }
}

void launch_glue_ratios(const RefineParams& r, double* out, hipStream_t st) {
  int n = (r.Hc / r.s) * r.bwc;
  hipLaunchKernelGGL(k_glue_ratios, dim3((n + 127) / 128), dim3(128), 0, st, r, out);
}

__device__ double interp_w(int n, double t, int* i0) {
  int i = (int)floor(t);
  if (i < 0) i = 0;
  if (i > n - 2) i = n - 2;
  *i0 = i;
  return t - i;
}

__global__ void k_interp(const double* fc, int Hc, int Wc, double* fa, double* fb, int Hf,
                         int Wf) {
  long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)Hf * Wf) return;
  int r = (int)(i / Wf), c = (int)(i % Wf);
  int r0, c0;
  double tr = interp_w(Hc, r * 0.5 - 0.25, &r0);
  double tc = interp_w(Wc, c * 0.5 - 0.25, &c0);
  double v00 = fc[(long long)r0 * Wc + c0], v01 = fc[(long long)r0 * Wc + c0 + 1];
  double v10 = fc[(long long)(r0 + 1) * Wc + c0], v11 = fc[(long long)(r0 + 1) * Wc + c0 + 1];
  double v = (1 - tr) * ((1 - tc) * v00 + tc * v01) + tr * ((1 - tc) * v10 + tc * v11);
  fa[i] = v;
  fb[i] = v;
}

void launch_interp(const double* fglued_c, int Hc, int Wc, double* fa, double* fb, int Hf,
                   int Wf, hipStream_t st) {
  long long n = (long long)Hf * Wf;
  hipLaunchKernelGGL(k_interp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, fglued_c, Hc,
                     Wc, fa, fb, Hf, Wf);
}

}  // namespace ddk

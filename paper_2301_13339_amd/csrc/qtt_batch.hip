// Batched form: thousands of independent lines (a1-a6 per line) in a few
// launches, captured in one hipGraph.
//
// Stages, each one launch over the whole batch:
//   1. k_batch_decompose (GEN 0): the signal of every line -> F (TT-SVD, eps,
//      rank cap), one persistent workgroup per line at a time;
//   2. k_batch_decompose (GEN 1): the sinc generator of every line (its own
//      bandwidth) -> W (d+1 modes, eps_w);
//   3. k_batch_full: f = full(F) for every line;
//   4. k_batch_toep, one launch per chunk of CB bits: y = T(w) f exactly, the
//      Toeplitz operator in QTT-matrix form applied to the full vector with
//      the state of CB consecutive bits in LDS (the state between chunks is
//      kept in HBM, overwritten in place);
//   5. k_batch_decompose (GEN 0) of y -> Z (the rounding: TT-SVD of the
//      represented tensor);
//   6. k_batch_full: out = full(Z).
// CB (chunk bits of stage 4) and the Full tile are chosen by timing the
// candidates on the batch itself the first time it runs.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "qtt_internal.hpp"

namespace qtt {

// one line of the batch (device table)
struct BatchLine {
  long long x_off;                     // sample offset in x / f / y / out
  long long f_core, w_core, z_core;    // core offsets (elements)
  long long st_off;                    // Toeplitz state offset (elements)
  int f_rank, w_rank, z_rank;          // rank array offsets
  int d;
};

__device__ __forceinline__ int find_line(const long long* start, int n, long long wg) {
  int lo = 0, hi = n - 1;  // last line with start <= wg
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= wg)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// capacity-strided offset of core k (0-based) for modes D and rank cap R
__device__ __forceinline__ long long core_off_dev(int D, int R, int k) {
  long long off = 0;
  int cprev = 1;
  for (int j = 0; j < k; ++j) {
    int c = R;
    if (j + 1 < 30 && (1 << (j + 1)) < c) c = 1 << (j + 1);
    if (D - j - 1 < 30 && (1 << (D - j - 1)) < c) c = 1 << (D - j - 1);
    if (j + 1 == D) c = 1;
    off += (long long)cprev * 2 * c;
    cprev = c;
  }
  return off;
}

// ======================================================== batched Full
// Workgroup = (line, block of high bits).  Positions split as lo (the first
// c bits), mid (the next hb bits) and the fixed top bits of the block:
//   out[lo + 2^c mid + 2^(c+hb) top] = sum_a Lam[lo][a] Rho[a][mid]
// with Lam the product of cores 1..c (2^c x r_c) and Rho the product of
// cores c+1..d with the top bits fixed (r_c x 2^hb).  Both are built in LDS
// one core at a time; each thread keeps its new entries in registers until
// every thread has read the old ones.
constexpr int kFullMaxLo = 128;   // 2^c
constexpr int kFullMaxMid = 64;   // 2^hb
constexpr int kFullMaxR = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_batch_full(const T* cores, const int32_t* ranks,
                                                    const BatchLine* lines, const long long* wg0,
                                                    int nlines, int which, int rcap, int cbits,
                                                    int hbits, T* out) {
  __shared__ double Lam[kFullMaxLo * kFullMaxR];
  __shared__ double Rho[kFullMaxR * kFullMaxMid];
  __shared__ double vtop[kFullMaxR];
  const int tid = threadIdx.x;
  const int l = find_line(wg0, nlines, blockIdx.x);
  const BatchLine ln = lines[l];
  const int d = ln.d;
  const long long coff = which == 0 ? ln.f_core : ln.z_core;
  const int32_t* rk = ranks + (which == 0 ? ln.f_rank : ln.z_rank);
  const int c = d < cbits ? d : cbits;
  const int hb = (d - c) < hbits ? (d - c) : hbits;
  const int top_bits = d - c - hb;
  const long long top = (long long)blockIdx.x - wg0[l];  // < 2^top_bits
  const T* G = cores + coff;
  // Lam: rows 2^k, cols r_k
  if (tid == 0) Lam[0] = 1.0;
  __syncthreads();
  for (int k = 1; k <= c; ++k) {
    const int r0 = rk[k - 1], r1 = rk[k];
    const int rows = 1 << k, half = rows >> 1;
    const T* Gk = G + core_off_dev(d, rcap, k - 1);
    double v[kFullMaxLo * kFullMaxR / 256];
#pragma unroll
    for (int t = 0; t < kFullMaxLo * kFullMaxR / 256; ++t) {
      const int e = tid + 256 * t;
      double s = 0.0;
      if (e < rows * r1) {
        const int row = e / r1, b = e - row * r1;
        const int i = row / half, lo = row - i * half;
        for (int a = 0; a < r0; ++a) s = fma(Lam[lo * r0 + a], (double)Gk[(a * 2 + i) * r1 + b], s);
      }
      v[t] = s;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kFullMaxLo * kFullMaxR / 256; ++t) {
      const int e = tid + 256 * t;
      if (e < rows * r1) Lam[e] = v[t];
    }
    __syncthreads();
  }
  // top part of the right chain: vector over the bond c + hb
  if (tid == 0) vtop[0] = 1.0;
  __syncthreads();
  for (int k = d; k > c + hb; --k) {
    const int r0 = rk[k - 1], r1 = rk[k];
    const int bit = (int)((top >> (k - c - hb - 1)) & 1);
    const T* Gk = G + core_off_dev(d, rcap, k - 1);
    double s = 0.0;
    if (tid < r0)
      for (int b = 0; b < r1; ++b) s = fma((double)Gk[(tid * 2 + bit) * r1 + b], vtop[b], s);
    __syncthreads();
    if (tid < r0) vtop[tid] = s;
    __syncthreads();
  }
  // Rho over the mid bits: Rho_k[a][i + 2 m] = sum_b G_k[a, i, b] Rho_{k+1}[b][m]
  const int rtop = rk[c + hb];
  for (int e = tid; e < rtop; e += 256) Rho[e] = vtop[e];
  __syncthreads();
  for (int k = c + hb; k > c; --k) {
    const int r0 = rk[k - 1], r1 = rk[k];
    const int cols = 1 << (c + hb - k + 1), hc = cols >> 1;
    const T* Gk = G + core_off_dev(d, rcap, k - 1);
    double v[kFullMaxR * kFullMaxMid / 256];
#pragma unroll
    for (int t = 0; t < kFullMaxR * kFullMaxMid / 256; ++t) {
      const int e = tid + 256 * t;
      double s = 0.0;
      if (e < r0 * cols) {
        const int a = e / cols, col = e - a * cols;
        const int i = col & 1, m = col >> 1;
        for (int b = 0; b < r1; ++b) s = fma((double)Gk[(a * 2 + i) * r1 + b], Rho[b * hc + m], s);
      }
      v[t] = s;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kFullMaxR * kFullMaxMid / 256; ++t) {
      const int e = tid + 256 * t;
      if (e < r0 * cols) Rho[e] = v[t];
    }
    __syncthreads();
  }
  // out tile
  const int rc = rk[c];
  const int nlo = 1 << c, nmid = 1 << hb;
  T* o = out + ln.x_off + (top << (c + hb));
  for (int e = tid; e < nlo * nmid; e += 256) {
    const int m = e >> c, lo = e & (nlo - 1);
    double s = 0.0;
    for (int a = 0; a < rc; ++a) s = fma(Lam[lo * rc + a], Rho[a * nmid + m], s);
    o[e] = (T)s;
  }
}

// ==================================================== batched Toeplitz
// One launch per chunk q of at most CB bits (chunk_of).  A workgroup takes
// one line and one value of the other bits; the state of
// the 2^cb positions for every bond (2 rho x 2^cb doubles) lives in LDS
// (double-buffered) across the cb steps, with the step rule of the
// single-signal Toeplitz product (binary adder with carry).  Between chunks
// the state is stored in HBM in the line's slot, layout [bond][position],
// overwritten in place (a workgroup reads all its positions before writing
// them, and workgroups own disjoint positions).
constexpr int kToepMaxBond = 48;  // 2 x the generator rank cap of the batch
constexpr int kToepMaxCB = 7;
constexpr int kToepPerWG = 32;    // values of the other bits per workgroup

// The d bits of a line split into nq = ceil(d / CB) chunks of nearly equal
// width (never narrower than d / nq), chunk q starting at bit b0.
__host__ __device__ inline bool chunk_of(int d, int CB, int q, int* b0, int* cb) {
  const int nq = (d + CB - 1) / CB;
  if (q >= nq) return false;
  const int base = d / nq, rem = d % nq;
  *cb = base + (q < rem ? 1 : 0);
  *b0 = q * base + (q < rem ? q : rem);
  return true;
}

template <typename T>
__global__ void __launch_bounds__(64) k_batch_toep(const T* wcores, const int32_t* ranks,
                                                   const BatchLine* lines, const long long* wg0,
                                                   int nlines, int wcap, int q, int CB,
                                                   int pmax, const T* f, T* state, T* y) {
  extern __shared__ double sm[];
  const int lane = threadIdx.x;
  const int l = find_line(wg0, nlines, blockIdx.x);
  const BatchLine ln = lines[l];
  const int d = ln.d;
  int b0, cb;
  if (!chunk_of(d, CB, q, &b0, &cb)) return;  // uniform: the line has no chunk q
  const int P = 1 << cb;
  const long long N = 1LL << d;
  const int32_t* wr = ranks + ln.w_rank;
  const T* W = wcores + ln.w_core;
  double* S0 = sm;
  double* S1 = sm + 2 * wcap * pmax;
  double* Ws = S1 + 2 * wcap * pmax;  // the core of the current step (rin x 2 x rout)
  // this workgroup takes kToepPerWG consecutive values of the other d - cb bits
  const long long nout = 1LL << (d - cb);
  const long long o_beg = ((long long)blockIdx.x - wg0[l]) * kToepPerWG;
  const long long o_end = (o_beg + kToepPerWG) < nout ? (o_beg + kToepPerWG) : nout;
  for (long long o = o_beg; o < o_end; ++o) {
  const long long lo = o & ((1LL << b0) - 1), hi = o >> b0;
  // load the state at bond b0 (the input vector when q == 0)
  const int rin0 = (q == 0) ? 1 : wr[b0];
  for (int e = lane; e < 2 * rin0 * P; e += 64) {
    const int b = e / P, p = e - b * P;
    const long long pos = lo | ((long long)p << b0) | (hi << (b0 + cb));
    double v;
    if (q == 0)
      v = (b == 1) ? (double)f[ln.x_off + pos] : 0.0;  // alpha = 0, carry-in 1
    else
      v = (double)state[ln.st_off + (long long)b * N + pos];
    S0[b * P + p] = v;
  }
  __syncthreads();
  double* cur = S0;
  double* nxt = S1;
  // One step: a work item is a pair of positions (p0, p1) that differ in the
  // step's bit (they share their inputs) and a group of 8 output bonds; per
  // item 4 rin loads of the state and ~32 rin FMAs.
  for (int j = 0; j < cb; ++j) {
    const int k = b0 + j + 1;  // 1-based bit
    const int rin = (k == 1) ? 1 : wr[k - 1];
    const int rout = wr[k];
    {
      // the core once into LDS: every work item reads all of it
      const T* Wk = W + core_off_dev(d + 1, wcap, k - 1);
      for (int e = lane; e < rin * 2 * rout; e += 64) Ws[e] = (double)Wk[e];
      __syncthreads();
    }
    const int half = 1 << j;
    const int npair = P >> 1;
    const int ngroup = (2 * rout + 7) >> 3;
    for (int it = lane; it < npair * ngroup; it += 64) {
      const int g = it / npair, pr = it - g * npair;
      const int p0 = ((pr >> j) << (j + 1)) | (pr & (half - 1));
      const int p1 = p0 | half;
      double acc[8][2];
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[t][0] = acc[t][1] = 0.0;
      for (int a = 0; a < rin; ++a) {
        double w[4][2];  // W_k[a, u, a1] for the group's 4 values of a1
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) {
          const int a1 = g * 4 + t2;
          w[t2][0] = a1 < rout ? Ws[(a * 2) * rout + a1] : 0.0;
          w[t2][1] = a1 < rout ? Ws[(a * 2 + 1) * rout + a1] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const double x0 = cur[(2 * a + c) * P + p0], x1 = cur[(2 * a + c) * P + p1];
#pragma unroll
          for (int t = 0; t < 8; ++t) {
            const int c1 = t & 1;
#pragma unroll
            for (int ob = 0; ob < 2; ++ob) {
#pragma unroll
              for (int n = 0; n < 2; ++n) {
                // forward product: output bit ob, input bit n
                const int v = ob + (1 - n) + c;
                if ((v >> 1) == c1) acc[t][ob] = fma(w[t >> 1][v & 1], n ? x1 : x0, acc[t][ob]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int bo = g * 8 + t;
        if (bo < 2 * rout) {
          nxt[bo * P + p0] = acc[t][0];
          nxt[bo * P + p1] = acc[t][1];
        }
      }
    }
    __syncthreads();
    double* tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  const int kend = b0 + cb;
  if (kend == d) {
    // contract the top carry with W_{d+1}: y = sum_{a,c} S[(a,c)] W_{d+1}[a, c, 0]
    const int rl = wr[d];
    const T* Wl = W + core_off_dev(d + 1, wcap, d);
    for (int p = lane; p < P; p += 64) {
      double s = 0.0;
      for (int b = 0; b < 2 * rl; ++b) s = fma(cur[b * P + p], (double)Wl[b], s);
      const long long pos = lo | ((long long)p << b0) | (hi << (b0 + cb));
      y[ln.x_off + pos] = (T)s;
    }
  } else {
    const int rout = wr[kend];
    for (int e = lane; e < 2 * rout * P; e += 64) {
      const int b = e / P, p = e - b * P;
      const long long pos = lo | ((long long)p << b0) | (hi << (b0 + cb));
      state[ln.st_off + (long long)b * N + pos] = (T)cur[b * P + p];
    }
  }
  __syncthreads();  // the LDS state is reused by the next value of the other bits
  }
}

__global__ void k_fill_i32(int32_t* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace qtt

// =============================================================== host plan
using namespace qtt;

struct qtt_batch {
  int n, dtype;
  double eps, eps_w;
  int f_rcap, w_rcap, z_rcap;
  std::vector<int32_t> d;
  std::vector<double> B;
  std::vector<int> order;  // lines by decreasing length (task order)
  std::vector<BatchLine> lines;
  std::vector<BatchTask> tf, tw, tz;
  std::vector<long long> full_wg0;                  // per line, for the Full tiles
  std::vector<std::vector<long long>> toep_wg0;     // per chunk
  std::vector<long long> toep_total;
  std::vector<int> toep_cbmax;                      // widest chunk of each pass
  long long full_total = 0;
  long long samples = 0, nmax = 0;
  int cb = 6, full_c = 7, full_hb = 6;
  int tuned = 0;
  // workspace layout (byte offsets)
  size_t o_lines, o_tf, o_tw, o_tz, o_fwg, o_twg, o_cnt, o_fcores, o_wcores, o_zcores, o_franks,
      o_wranks, o_zranks, o_status, o_f, o_y, o_state, o_scr, total;
  long long fcore_elems = 0, wcore_elems = 0, zcore_elems = 0;
  int nranks_f = 0, nranks_w = 0, nranks_z = 0;
  long long state_elems = 0;
  long long wstride = 0;
  int nwg = 256;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void* gx = nullptr;
  void* gout = nullptr;
  void* gws = nullptr;
  hipStream_t gstream = nullptr;
  int uploaded_for = 0;
  const void* up_ws = nullptr;
};

static int caps_of(int D, int R, int k) {
  if (k == 0 || k == D) return 1;
  int c = R;
  if (k < 30 && (1 << k) < c) c = 1 << k;
  if (D - k < 30 && (1 << (D - k)) < c) c = 1 << (D - k);
  return c;
}

static long long core_elems_dr(int D, int R) {
  long long e = 0;
  for (int k = 0; k < D; ++k) e += (long long)caps_of(D, R, k) * 2 * caps_of(D, R, k + 1);
  return e;
}

static void batch_layout(qtt_batch* p) {
  const int n = p->n;
  // tables
  p->lines.resize(n);
  p->tf.resize(n);
  p->tw.resize(n);
  p->tz.resize(n);
  long long xo = 0, fo = 0, wo = 0, zo = 0, so = 0;
  int fr = 0, wr = 0, zr = 0;
  std::vector<long long> xoff(n);
  for (int l = 0; l < n; ++l) {
    xoff[l] = xo;
    xo += 1LL << p->d[l];
  }
  p->samples = xo;
  p->nmax = 0;
  for (int l = 0; l < n; ++l) {
    const int d = p->d[l];
    BatchLine& L = p->lines[l];
    L.d = d;
    L.x_off = xoff[l];
    L.f_core = fo;
    fo += core_elems_dr(d, p->f_rcap);
    L.w_core = wo;
    wo += core_elems_dr(d + 1, p->w_rcap);
    L.z_core = zo;
    zo += core_elems_dr(d, p->z_rcap);
    L.f_rank = fr;
    fr += d + 1;
    L.w_rank = wr;
    wr += d + 2;
    L.z_rank = zr;
    zr += d + 1;
    L.st_off = so;
    so += (long long)(2 * p->w_rcap) << d;
    if ((2LL << d) > p->nmax) p->nmax = 2LL << d;  // generator has 2^(d+1) samples
  }
  p->fcore_elems = fo;
  p->wcore_elems = wo;
  p->zcore_elems = zo;
  p->nranks_f = fr;
  p->nranks_w = wr;
  p->nranks_z = zr;
  p->state_elems = so;
  // tasks in decreasing size (the persistent workgroups take them in order)
  p->order.resize(n);
  std::iota(p->order.begin(), p->order.end(), 0);
  std::stable_sort(p->order.begin(), p->order.end(),
                   [&](int a, int b) { return p->d[a] > p->d[b]; });
  for (int i = 0; i < n; ++i) {
    const int l = p->order[i];
    const BatchLine& L = p->lines[l];
    BatchTask t{};
    t.x_off = L.x_off;
    t.core_off = L.f_core;
    t.rank_off = L.f_rank;
    t.status_idx = l;
    t.D = L.d;
    t.rcap = p->f_rcap;
    t.nk = 0;
    t.B = 0.0;
    t.eps = p->eps;
    p->tf[i] = t;
    t.core_off = L.w_core;
    t.rank_off = L.w_rank;
    t.status_idx = n + l;
    t.D = L.d + 1;
    t.rcap = p->w_rcap;
    t.nk = L.d;
    t.B = p->B[l];
    t.eps = p->eps_w;
    p->tw[i] = t;
    t.core_off = L.z_core;
    t.rank_off = L.z_rank;
    t.status_idx = 2 * n + l;
    t.D = L.d;
    t.rcap = p->z_rcap;
    t.nk = 0;
    t.B = 0.0;
    t.eps = p->eps;
    p->tz[i] = t;
  }
}

static void batch_grids(qtt_batch* p) {
  const int n = p->n;
  p->full_wg0.resize(n);
  long long acc = 0;
  for (int l = 0; l < n; ++l) {
    p->full_wg0[l] = acc;
    const int d = p->d[l];
    const int c = std::min(d, p->full_c);
    const int hb = std::min(d - c, p->full_hb);
    acc += 1LL << (d - c - hb);
  }
  p->full_total = acc;
  int maxd = 0;
  for (int l = 0; l < n; ++l) maxd = std::max(maxd, (int)p->d[l]);
  const int nq = (maxd + p->cb - 1) / p->cb;
  p->toep_wg0.assign(nq, std::vector<long long>(n));
  p->toep_total.assign(nq, 0);
  p->toep_cbmax.assign(nq, 0);
  for (int qi = 0; qi < nq; ++qi) {
    long long a = 0;
    for (int l = 0; l < n; ++l) {
      p->toep_wg0[qi][l] = a;
      int b0, cbl;
      if (chunk_of(p->d[l], p->cb, qi, &b0, &cbl)) {
        a += ((1LL << (p->d[l] - cbl)) + kToepPerWG - 1) / kToepPerWG;
        p->toep_cbmax[qi] = std::max(p->toep_cbmax[qi], cbl);
      }
    }
    p->toep_total[qi] = a;
  }
}

static void batch_ws(qtt_batch* p) {
  const size_t es = elem_size(p->dtype);
  const int n = p->n;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += bytes;
    return o;
  };
  p->o_lines = take(sizeof(BatchLine) * n);
  p->o_tf = take(sizeof(BatchTask) * n);
  p->o_tw = take(sizeof(BatchTask) * n);
  p->o_tz = take(sizeof(BatchTask) * n);
  p->o_fwg = take(sizeof(long long) * n);
  int maxd = 0;
  for (int l = 0; l < n; ++l) maxd = std::max(maxd, (int)p->d[l]);
  const int nq_max = (maxd + 4) / 5 + 1;  // room for any candidate chunk width >= 5
  p->o_twg = take(sizeof(long long) * (size_t)n * nq_max);
  p->o_cnt = take(sizeof(int32_t) * 8);
  p->o_fcores = take(es * p->fcore_elems);
  p->o_wcores = take(es * p->wcore_elems);
  p->o_zcores = take(es * p->zcore_elems);
  p->o_franks = take(sizeof(int32_t) * p->nranks_f);
  p->o_wranks = take(sizeof(int32_t) * p->nranks_w);
  p->o_zranks = take(sizeof(int32_t) * p->nranks_z);
  p->o_status = take(sizeof(int32_t) * 3 * n);
  p->o_f = take(es * p->samples);
  p->o_y = take(es * p->samples);
  p->o_state = take(es * p->state_elems);
  p->wstride = (long long)(((size_t)batch_wg_doubles() * 8 + 2 * es * p->nmax + 255) & ~size_t(255));
  p->o_scr = take((size_t)p->wstride * p->nwg);
  p->total = (off + 255) & ~size_t(255);
}

static int batch_upload(qtt_batch* p, char* ws, hipStream_t s) {
  const int n = p->n;
  QTT_HIP_CHECK(hipMemcpyAsync(ws + p->o_lines, p->lines.data(), sizeof(BatchLine) * n,
                               hipMemcpyHostToDevice, s));
  QTT_HIP_CHECK(hipMemcpyAsync(ws + p->o_tf, p->tf.data(), sizeof(BatchTask) * n,
                               hipMemcpyHostToDevice, s));
  QTT_HIP_CHECK(hipMemcpyAsync(ws + p->o_tw, p->tw.data(), sizeof(BatchTask) * n,
                               hipMemcpyHostToDevice, s));
  QTT_HIP_CHECK(hipMemcpyAsync(ws + p->o_tz, p->tz.data(), sizeof(BatchTask) * n,
                               hipMemcpyHostToDevice, s));
  QTT_HIP_CHECK(hipMemcpyAsync(ws + p->o_fwg, p->full_wg0.data(), sizeof(long long) * n,
                               hipMemcpyHostToDevice, s));
  for (size_t qi = 0; qi < p->toep_wg0.size(); ++qi)
    QTT_HIP_CHECK(hipMemcpyAsync(ws + p->o_twg + sizeof(long long) * n * qi,
                                 p->toep_wg0[qi].data(), sizeof(long long) * n,
                                 hipMemcpyHostToDevice, s));
  // tables are read by later kernels on the same stream; the host vectors
  // live in the plan, so the asynchronous copies stay valid
  return QTT_OK;
}

template <typename T>
static int batch_stages(qtt_batch* p, const T* x, T* out, char* ws, hipStream_t s) {
  const int n = p->n;
  const BatchLine* lines = reinterpret_cast<const BatchLine*>(ws + p->o_lines);
  int32_t* cnt = reinterpret_cast<int32_t*>(ws + p->o_cnt);
  int32_t* status = reinterpret_cast<int32_t*>(ws + p->o_status);
  T* fc = reinterpret_cast<T*>(ws + p->o_fcores);
  T* wc = reinterpret_cast<T*>(ws + p->o_wcores);
  T* zc = reinterpret_cast<T*>(ws + p->o_zcores);
  int32_t* fr = reinterpret_cast<int32_t*>(ws + p->o_franks);
  int32_t* wr = reinterpret_cast<int32_t*>(ws + p->o_wranks);
  int32_t* zr = reinterpret_cast<int32_t*>(ws + p->o_zranks);
  T* f = reinterpret_cast<T*>(ws + p->o_f);
  T* y = reinterpret_cast<T*>(ws + p->o_y);
  T* st = reinterpret_cast<T*>(ws + p->o_state);
  char* scr = ws + p->o_scr;
  const long long* fwg = reinterpret_cast<const long long*>(ws + p->o_fwg);
  // counters and status words start at zero (fill kernels, not memsets, so
  // the sequence can be captured in a graph)
  {
    ProbeScope _ps(QTT_K_OTHER, s);
    k_fill_i32<<<1, 64, 0, s>>>(cnt, 8, 0);
    QTT_LAUNCH_CHECK();
    k_fill_i32<<<(3 * n + 255) / 256, 256, 0, s>>>(status, 3 * n, 0);
    QTT_LAUNCH_CHECK();
  }
  const int dt = p->dtype;
  int rc = run_batch_decompose(dt, 0, x, reinterpret_cast<const BatchTask*>(ws + p->o_tf), n,
                               cnt + 0, fc, fr, status, scr, p->wstride, p->nmax, p->nwg, s);
  if (rc) return rc;
  rc = run_batch_decompose(dt, 1, nullptr, reinterpret_cast<const BatchTask*>(ws + p->o_tw), n,
                           cnt + 1, wc, wr, status, scr, p->wstride, p->nmax, p->nwg, s);
  if (rc) return rc;
  {
    ProbeScope _ps(QTT_K_BATCH, s);
    k_batch_full<T><<<(unsigned)p->full_total, 256, 0, s>>>(fc, fr, lines, fwg, n, 0, p->f_rcap,
                                                             p->full_c, p->full_hb, f);
    QTT_LAUNCH_CHECK();
    const size_t lds_max =
        sizeof(double) * (2 * kToepMaxBond * (1 << kToepMaxCB) + kToepMaxBond * kToepMaxBond);
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [lds_max] {
      set_lds_limit((const void*)k_batch_toep<T>, (int)lds_max, &attr_err);
    });
    QTT_HIP_CHECK(attr_err);
    for (size_t qi = 0; qi < p->toep_wg0.size(); ++qi) {
      if (p->toep_total[qi] > 0xFFFFFFFFLL / 64) return QTT_ENOTSUP;  // grid limit
      const long long* twg = reinterpret_cast<const long long*>(ws + p->o_twg) + (size_t)n * qi;
      const int pmax = 1 << p->toep_cbmax[qi];
      const size_t lds =
          sizeof(double) * (2 * (2 * p->w_rcap) * pmax + p->w_rcap * 2 * p->w_rcap);
      k_batch_toep<T><<<(unsigned)p->toep_total[qi], 64, lds, s>>>(
          wc, wr, lines, twg, n, p->w_rcap, (int)qi, p->cb, pmax, f, st, y);
      QTT_LAUNCH_CHECK();
    }
  }
  rc = run_batch_decompose(dt, 0, y, reinterpret_cast<const BatchTask*>(ws + p->o_tz), n,
                           cnt + 2, zc, zr, status, scr, p->wstride, p->nmax, p->nwg, s);
  if (rc) return rc;
  {
    ProbeScope _ps(QTT_K_BATCH, s);
    k_batch_full<T><<<(unsigned)p->full_total, 256, 0, s>>>(zc, zr, lines, fwg, n, 1, p->z_rcap,
                                                             p->full_c, p->full_hb, out);
    QTT_LAUNCH_CHECK();
  }
  return QTT_OK;
}

static int batch_launch(qtt_batch* p, const void* x, void* out, char* ws, hipStream_t s) {
  if (p->dtype == QTT_F64)
    return batch_stages<double>(p, static_cast<const double*>(x), static_cast<double*>(out), ws,
                                s);
  return batch_stages<float>(p, static_cast<const float*>(x), static_cast<float*>(out), ws, s);
}

// Chunk width of the Toeplitz stage: time each candidate on the batch (the
// whole pipeline, so the chunk layout of the state is exercised end to end)
// and keep the fastest.  Runs once per plan, before any graph capture.
static int batch_tune(qtt_batch* p, const void* x, void* out, char* ws, hipStream_t s) {
  const int cands[3] = {5, 6, 7};
  float best = 1e30f;
  int bestcb = p->cb;
  hipEvent_t e0, e1;
  QTT_HIP_CHECK(hipEventCreate(&e0));
  QTT_HIP_CHECK(hipEventCreate(&e1));
  int rc = QTT_OK;
  for (int ci = 0; ci < 3 && rc == QTT_OK; ++ci) {
    p->cb = cands[ci];
    batch_grids(p);
    rc = batch_upload(p, ws, s);
    if (rc) break;
    rc = batch_launch(p, x, out, ws, s);  // warm-up
    if (rc) break;
    (void)hipEventRecord(e0, s);
    rc = batch_launch(p, x, out, ws, s);
    if (rc) break;
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) {
      rc = QTT_EHIP;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      bestcb = cands[ci];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  p->cb = bestcb;
  batch_grids(p);
  p->tuned = 1;
  return batch_upload(p, ws, s);
}

extern "C" {

int qtt_batch_create(int n_lines, const int32_t* d, const double* B, int dtype, double eps,
                     int max_rank, double eps_w, int w_max_rank, int round_max_rank,
                     qtt_batch** plan, size_t* ws_bytes) {
  if (n_lines < 1 || !d || !B || !plan || (dtype != QTT_F32 && dtype != QTT_F64) ||
      !(eps >= 0.0) || !isfinite(eps) || !(eps_w >= 0.0) || !isfinite(eps_w) || max_rank < 0 ||
      max_rank > QTT_MAX_RANK || w_max_rank < 0 || round_max_rank < 0 ||
      round_max_rank > QTT_MAX_RANK)
    return QTT_EINVAL;
  const int wr = w_max_rank == 0 ? 16 : w_max_rank;
  if (wr > kToepMaxBond / 2) return QTT_ENOTSUP;
  for (int l = 0; l < n_lines; ++l) {
    if (d[l] < 1 || d[l] > QTT_BATCH_MAXD) return QTT_EINVAL;
    if (!(B[l] > 0.0) || !isfinite(B[l])) return QTT_EINVAL;
  }
  qtt_batch* p = new (std::nothrow) qtt_batch();
  if (!p) return QTT_ENOTSUP;
  p->n = n_lines;
  p->dtype = dtype;
  p->eps = eps;
  p->eps_w = eps_w;
  p->f_rcap = max_rank == 0 ? kMaxRank : max_rank;
  p->w_rcap = wr;
  p->z_rcap = round_max_rank == 0 ? kMaxRank : round_max_rank;
  p->d.assign(d, d + n_lines);
  p->B.assign(B, B + n_lines);
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
      ncu = prop.multiProcessorCount;
  }
  p->nwg = std::min(ncu, n_lines);
  batch_layout(p);
  batch_grids(p);
  batch_ws(p);
  *plan = p;
  if (ws_bytes) *ws_bytes = p->total;
  return QTT_OK;
}

int qtt_batch_destroy(qtt_batch* plan) {
  if (!plan) return QTT_EINVAL;
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  delete plan;
  return QTT_OK;
}

int qtt_batch_run(qtt_batch* plan, const void* x, void* out, void* ws, size_t ws_bytes,
                  int use_graph, void* stream) {
  if (!plan || !x || !out || !ws) return QTT_EINVAL;
  if (ws_bytes < plan->total) return QTT_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(ws);
  if (!plan->tuned || plan->up_ws != ws) {
    const int rc = plan->tuned ? batch_upload(plan, w, s) : batch_tune(plan, x, out, w, s);
    if (rc) return rc;
    plan->up_ws = ws;
  }
  if (!use_graph) return batch_launch(plan, x, out, w, s);
  if (!plan->exec || plan->gx != x || plan->gout != out || plan->gws != ws ||
      plan->gstream != s) {
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    plan->exec = nullptr;
    plan->graph = nullptr;
    // capture on a stream of our own (the legacy default stream cannot be
    // captured); capturing only records the launches, nothing runs here
    hipStream_t cs = nullptr;
    QTT_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    const hipError_t eb = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
      (void)hipStreamDestroy(cs);
      set_hip_error(eb);
      return QTT_EHIP;
    }
    const int rc = batch_launch(plan, x, out, w, cs);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) {
      set_hip_error(ec);
      return QTT_EHIP;
    }
    plan->graph = g;
    QTT_HIP_CHECK(hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
    plan->gx = x;
    plan->gout = out;
    plan->gws = ws;
    plan->gstream = s;
  }
  QTT_HIP_CHECK(hipGraphLaunch(plan->exec, s));
  return QTT_OK;
}

int qtt_batch_info(const qtt_batch* plan, int line, int which, int64_t* rank_off_bytes,
                   int64_t* core_off_bytes, int32_t* rank_cap, int64_t* sample_off) {
  if (!plan || line < 0 || line >= plan->n || which < 0 || which > 2) return QTT_EINVAL;
  const BatchLine& L = plan->lines[line];
  const size_t es = elem_size(plan->dtype);
  int64_t ro = 0, co = 0;
  int cap = 0;
  if (which == 0) {
    ro = plan->o_franks + sizeof(int32_t) * L.f_rank;
    co = plan->o_fcores + es * L.f_core;
    cap = plan->f_rcap;
  } else if (which == 1) {
    ro = plan->o_wranks + sizeof(int32_t) * L.w_rank;
    co = plan->o_wcores + es * L.w_core;
    cap = plan->w_rcap;
  } else {
    ro = plan->o_zranks + sizeof(int32_t) * L.z_rank;
    co = plan->o_zcores + es * L.z_core;
    cap = plan->z_rcap;
  }
  if (rank_off_bytes) *rank_off_bytes = ro;
  if (core_off_bytes) *core_off_bytes = co;
  if (rank_cap) *rank_cap = cap;
  if (sample_off) *sample_off = L.x_off;
  return QTT_OK;
}

int qtt_batch_status_offset(const qtt_batch* plan, int64_t* status_off_bytes, int32_t* chunk_bits) {
  if (!plan) return QTT_EINVAL;
  if (status_off_bytes) *status_off_bytes = (int64_t)plan->o_status;
  if (chunk_bits) *chunk_bits = plan->cb;
  return QTT_OK;
}

}  // extern "C"

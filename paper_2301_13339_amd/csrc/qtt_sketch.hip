// Randomised rounding (the precision form): the TT-SVD sweep of a full
// vector in which every truncated SVD is taken by the randomised range
// finder and RSVD (Algorithms 4 and 5, Appendix A).
//
// Step k works on the remainder X_k (n x m row-major, m = 2 r_{k-1}; the
// unfolding is A = X_k^T):
//   1. one streaming pass forms Y = A Omega (m x ell) -- the sketch GEMM, in
//      FP32 or with BF16-rounded operands, FP32 accumulation, FP64 combine
//      of the per-block partials -- and the Gram G = A A^T (FP64);
//   2. one workgroup: Q = qr(Y) (FP64 Householder, ell' = min(m, ell)
//      columns), B B^T = Q^T G Q, its eigendecomposition gives sigma(B) and
//      U~, the rank rule of Algorithm 1 picks r, U = Q U~_r is core k;
//   3. X_{k+1} = X_k U read as (n/2) x 2r (the remainder Sigma V^T = U^T A).
// Omega[row][col] of step k is one standard normal from Philox-4x32-10 with
// counter (row, col, k, 0) and key (seed low, seed high) through the
// Box-Muller transform of its first two words.
#include <math.h>

#include <mutex>

#include "qtt_eig.hpp"
#include "qtt_internal.hpp"
#include "qtt_philox.hpp"

namespace qtt {

// round to the nearest bfloat16 (ties to even) and back
__device__ __forceinline__ float bf16_round(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) != 0x7F800000u) u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// ------------------------------------------------------ Gram + sketch pass
// Partials per block: G (m x m, FP64) then Y (m x ell, FP32 sums stored as
// doubles), row stride pstride.  Thread (ty, tx) owns the TS x TS tile of G
// at rows ty*TS.., cols tx*TS.. and the TS x 4 tile of Y at rows ty*TS..,
// cols tx*4.. (ell <= 64).
constexpr int kSkSR = 32;
constexpr int kSkMaxEll = 64;

template <typename T, int BF, int TS>
__global__ void __launch_bounds__(256) k_gram_sketch(const T* X, long long n, const int32_t* ranks,
                                                     int kin, int ell, uint32_t key0,
                                                     uint32_t key1, int step, double* partials,
                                                     int pstride) {
  extern __shared__ double smem[];
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  // with ell >= m the range finder spans all of R^m whatever Omega is (the
  // step is the exact SVD): only the Gram is formed
  if (m <= ell) ell = 0;
  double* Xs = smem;                                     // kSkSR x m
  float* Os = reinterpret_cast<float*>(Xs + kSkSR * m);  // kSkSR x ell
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  double g[TS][TS];
  float y[TS][4];
#pragma unroll
  for (int a = 0; a < TS; ++a) {
#pragma unroll
    for (int b = 0; b < TS; ++b) g[a][b] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) y[a][b] = 0.f;
  }
  const long long nstage = (n + kSkSR - 1) / kSkSR;
  for (long long sidx = blockIdx.x; sidx < nstage; sidx += gridDim.x) {
    const long long r0 = sidx * kSkSR;
    const int nr = (int)((n - r0) < kSkSR ? (n - r0) : kSkSR);
    for (int e = tid; e < kSkSR * m; e += 256) Xs[e] = (e / m < nr) ? (double)X[r0 * m + e] : 0.0;
    for (int e = tid; e < kSkSR * ell; e += 256) {
      const int rr = e / ell, c = e - rr * ell;
      float o = 0.f;
      if (rr < nr) {
        o = (float)omega_entry(r0 + rr, c, step, key0, key1);
        if (BF) o = bf16_round(o);
      }
      Os[e] = o;
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const double* xr = Xs + rr * m;
      double xa[TS], xb[TS];
      float xs[TS];
#pragma unroll
      for (int a = 0; a < TS; ++a) {
        const int i = ty * TS + a;
        xa[a] = i < m ? xr[i] : 0.0;
        xs[a] = BF ? bf16_round((float)xa[a]) : (float)xa[a];
      }
#pragma unroll
      for (int b = 0; b < TS; ++b) {
        const int j = tx * TS + b;
        xb[b] = j < m ? xr[j] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < TS; ++a)
#pragma unroll
        for (int b = 0; b < TS; ++b) g[a][b] = fma(xa[a], xb[b], g[a][b]);
      float ob[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int c = tx * 4 + b;
        ob[b] = c < ell ? Os[rr * ell + c] : 0.f;
      }
#pragma unroll
      for (int a = 0; a < TS; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) y[a][b] = fmaf(xs[a], ob[b], y[a][b]);
    }
    __syncthreads();
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int a = 0; a < TS; ++a) {
    const int i = ty * TS + a;
    if (i >= m) continue;
#pragma unroll
    for (int b = 0; b < TS; ++b) {
      const int j = tx * TS + b;
      if (j < m) P[i * m + j] = g[a][b];
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = tx * 4 + b;
      if (c < ell) P[m * m + i * ell + c] = (double)y[a][b];
    }
  }
}

// The Gram alone for narrow remainders (m <= 16, and m <= ell so that no
// sketch is needed): thread t accumulates entry (i, j) of G over the rows
// g, g + Gr, ... of each 2048-value stage (g = t / m^2, Gr = 256 / m^2 row
// groups), so all threads work however small m is; the groups are summed in
// a fixed order at the end.
template <typename T>
__global__ void __launch_bounds__(256) k_gram_small(const T* X, long long n, const int32_t* ranks,
                                                    int kin, double* partials, int pstride) {
  constexpr int SV = 2048;
  __shared__ double Xs[SV];
  __shared__ double red[256];
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  const int m2 = m * m, Gr = 256 / m2;
  const int tid = threadIdx.x, g = tid / m2, e = tid - g * m2, i = e / m, j = e - i * m;
  const bool act = g < Gr;
  const int SRs = SV / m;  // rows per stage
  const long long nstage = (n + SRs - 1) / SRs;
  double acc = 0.0;
  for (long long sidx = blockIdx.x; sidx < nstage; sidx += gridDim.x) {
    const long long r0 = sidx * SRs;
    const int nr = (int)((n - r0) < SRs ? (n - r0) : SRs);
    __syncthreads();
    for (int q = tid; q < nr * m; q += 256) Xs[q] = (double)X[r0 * m + q];
    __syncthreads();
    if (act) {
#pragma unroll 4
      for (int rr = g; rr < nr; rr += Gr) acc = fma(Xs[rr * m + i], Xs[rr * m + j], acc);
    }
  }
  red[tid] = act ? acc : 0.0;
  __syncthreads();
  if (tid < m2) {
    double sum = 0.0;
    for (int gg = 0; gg < Gr; ++gg) sum += red[gg * m2 + tid];
    partials[(size_t)blockIdx.x * pstride + tid] = sum;  // entry i*m + j
  }
}

// out[e] = sum over the partials of entry e (fixed order)
__global__ void k_sum_partials(const double* partials, int pstride, int nparts,
                               const int32_t* ranks, int kin, int ell, double* out) {
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  const int count = m * m + (m > ell ? m * ell : 0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  // eight independent loads in flight, summed in a fixed order
  double s = 0.0;
  int b = 0;
  for (; b + 7 < nparts; b += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = partials[(size_t)(b + u) * pstride + e];
    s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  }
  for (; b < nparts; ++b) s += partials[(size_t)b * pstride + e];
  out[e] = s;
}

// ---------------------------------------------------------- the small step
// From G and Y of step k (in gy): Q = qr(Y), H = Q^T G Q, eigen + rank rule,
// U = Q U~_r -> core k and umat (m x r).  With first != 0 also the norm of
// the tensor (trace of G) and tau^2 into scal.  gT: m x ell doubles.
template <typename T>
__global__ void __launch_bounds__(kEigThreads) k_sketch_step(
    const double* gy, int k, int D, double eps, int first, int ell, double* scal, int cap_k,
    T* cores, long long off_k, double* umat, double* gT, StepOut so) {
  constexpr int NT = kEigThreads, LDA = kEigLds + 1, LQ = kSkMaxEll + 1;
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG16 = NT / 16;
  const int rp = (k == 1) ? 1 : so.ranks[k - 1];
  const int m = 2 * rp;
  const int el = ell < m ? ell : m;  // ell'
  const double* G = gy;
  const double* Yg = gy + m * m;
  double* Qs = smem;                    // m x LQ (Y, then the reflectors, then Q)
  double* A = Qs + kMaxM * LQ;          // LDA x LDA
  double* V = A + LDA * LDA;            // LDA x LDA
  double* lam = V + LDA * LDA;          // 72
  double* sx = lam + 72;                // kEigScratch
  double* bt = sx + kEigScratch;        // kSkMaxEll
  int* perm = (int*)(bt + kSkMaxEll);   // 72
  int* iscr = perm + 72;                // 8
  if (first && tid == 0) {
    double nrm2 = 0.0;
    for (int i = 0; i < m; ++i) nrm2 += G[i * m + i];
    scal[0] = nrm2;
    scal[1] = (D > 1) ? eps * eps * nrm2 / (double)(D - 1) : 0.0;
    so.ranks[0] = 1;
  }
  // ell >= m: the range of Y is all of R^m (Q square), so H = Q^T G Q is
  // similar to G and U = Q U~ are G's eigenvectors: the exact step on G
  const bool full = el == m;
  if (!full) {
    for (int e = tid; e < m * el; e += NT) {
      const int i = e / el, j = e - i * el;
      Qs[i * LQ + j] = Yg[i * ell + j];
    }
  } else {
    for (int e = tid; e < m * m; e += NT) {
      const int i = e / m, j = e - i * m;
      A[i * LDA + j] = G[e];
    }
  }
  __threadfence();
  __syncthreads();
  const double tau2 = scal[1];
  // Householder QR of Y (m x el); reflector j overwrites column j (rows j..)
  for (int j = 0; !full && j < el; ++j) {
    double xs = 0.0;
    for (int i = j + (tid & 63); i < m; i += 64) xs = fma(Qs[i * LQ + j], Qs[i * LQ + j], xs);
    xs = sum64(xs);
    const double x0 = Qs[j * LQ + j];
    const double alpha = sqrt(xs);
    double beta = 0.0, v0 = 1.0;
    if (alpha > 0.0) {
      const double sg = x0 >= 0.0 ? 1.0 : -1.0;
      v0 = x0 + sg * alpha;
      beta = 2.0 / (xs - x0 * x0 + v0 * v0);
    }
    __syncthreads();
    if (tid == 0) {
      Qs[j * LQ + j] = v0;
      bt[j] = beta;
    }
    __syncthreads();
    // apply H_j to columns j+1..el-1
    for (int c = j + 1 + g16; c < el; c += NG16) {
      double d = 0.0;
      for (int i = j + l16; i < m; i += 16) d = fma(Qs[i * LQ + j], Qs[i * LQ + c], d);
      d = sum16(d) * beta;
      for (int i = j + l16; i < m; i += 16) Qs[i * LQ + c] -= d * Qs[i * LQ + j];
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{el-1} [I; 0], formed in place from the last reflector
  for (int j = el - 1; !full && j >= 0; --j) {
    const double beta = bt[j];
    for (int c = j + 1 + g16; c < el; c += NG16) {
      double d = 0.0;
      for (int i = j + l16; i < m; i += 16) d = fma(Qs[i * LQ + j], Qs[i * LQ + c], d);
      d = sum16(d) * beta;
      for (int i = j + l16; i < m; i += 16) Qs[i * LQ + c] -= d * Qs[i * LQ + j];
    }
    __syncthreads();
    // column j = H_j e_j
    const double vj = Qs[j * LQ + j];
    __syncthreads();
    for (int i = tid; i < m; i += NT) {
      double q;
      if (i < j)
        q = 0.0;
      else if (i == j)
        q = 1.0 - beta * vj * vj;
      else
        q = -beta * vj * Qs[i * LQ + j];
      Qs[i * LQ + j] = q;
    }
    __syncthreads();
  }
  // T1 = G Q (m x el) into gT, then H = Q^T T1 (el x el) into A
  for (int e = tid; !full && e < m * el; e += NT) {
    const int i = e / el, b = e - i * el;
    double s = 0.0;
    for (int j2 = 0; j2 < m; ++j2) s = fma(G[i * m + j2], Qs[j2 * LQ + b], s);
    gT[e] = s;
  }
  __threadfence();
  __syncthreads();
  for (int e = tid; !full && e < el * el; e += NT) {
    const int a = e / el, b = e - a * el;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(Qs[i * LQ + a], gT[i * el + b], s);
    A[a * LDA + b] = s;
  }
  __syncthreads();
  // symmetrise (rounding) and solve
  for (int e = tid; e < el * el; e += NT) {
    const int a = e / el, b = e - a * el;
    if (a < b) {
      const double s = 0.5 * (A[a * LDA + b] + A[b * LDA + a]);
      A[a * LDA + b] = s;
      A[b * LDA + a] = s;
    }
  }
  __syncthreads();
  const int r = solve_and_truncate<NT>(lds(A), lds(V), el, LDA, lds(sx), lds(iscr), lds(lam),
                                       lds(perm), tau2, cap_k, k, so);
  // U = Q V_r (m x r)
  for (int e = tid; e < m * r; e += NT) {
    const int i = e / r, b = e - i * r;
    double s = 0.0;
    if (full) {
      s = V[i * LDA + b];
    } else {
      for (int a = 0; a < el; ++a) s = fma(Qs[i * LQ + a], V[a * LDA + b], s);
    }
    umat[e] = s;
    // core k: (a, i, b) <- U[a + rp*i][b]
    const int ii = i / rp, aa = i - ii * rp;
    cores[off_k + (long long)(aa * 2 + ii) * r + b] = (T)s;
  }
}

// X_{k+1} = X_k U (n x r), written row-major (read as (n/2) x 2r next)
template <typename T>
__global__ void __launch_bounds__(256) k_sketch_project(const T* X, long long n,
                                                        const int32_t* ranks, int kin, int kout,
                                                        const double* U, T* Xout) {
  __shared__ double Us[kMaxM * kMaxRank];
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  const int r = ranks[kout];
  for (int e = threadIdx.x; e < m * r; e += 256) Us[e] = U[e];
  __syncthreads();
  const long long total = n * r;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (long long)gridDim.x * 256) {
    const long long row = e / r;
    const int b = (int)(e - row * r);
    double s = 0.0;
    for (int c = 0; c < m; ++c) s = fma((double)X[row * m + c], Us[c * r + b], s);
    Xout[e] = (T)s;
  }
}

// last core (r_{D-1}, 2, 1): core[a*2 + i] = X_D[a + r i]
template <typename T>
__global__ void k_sketch_last(const T* X, const int32_t* ranks, int D, T* cores, long long off,
                              int32_t* ranks_out) {
  const int r = ranks[D - 1];
  for (int e = threadIdx.x; e < 2 * r; e += blockDim.x) {
    const int a = e >> 1, i = e & 1;
    cores[off + e] = X[a + r * i];
  }
  if (threadIdx.x == 0) ranks_out[D] = 1;
}

// ------------------------------------------------------------------ host
size_t sketch_step_lds() {
  const int LDA = kEigLds + 1, LQ = kSkMaxEll + 1;
  return sizeof(double) * ((size_t)kMaxM * LQ + 2 * LDA * LDA + 72 + kEigScratch + kSkMaxEll) +
         sizeof(int) * (72 + 8 + 256);
}

struct SketchPlan {
  double* scal;
  double* partials;
  int pstride;
  double* gy;
  double* gT;
  double* umat;
  void* xbuf[2];
  size_t bytes;
};

static void sketch_plan(int D, int dtype, int ell, void* ws, SketchPlan* p) {
  Arena ar(ws);
  const size_t es = elem_size(dtype);
  p->scal = ar.take<double>(16);
  p->pstride = kMaxM * kMaxM + kMaxM * ell;
  p->partials = ar.take<double>((size_t)kMaxPartials * p->pstride);
  p->gy = ar.take<double>((size_t)p->pstride);
  p->gT = ar.take<double>((size_t)kMaxM * kSkMaxEll);
  p->umat = ar.take<double>((size_t)kMaxM * kMaxRank);
  const size_t N = (size_t)1 << D;
  p->xbuf[0] = ar.take<char>(N * es);
  p->xbuf[1] = ar.take<char>(N * es);
  p->bytes = ar.size();
}

size_t sketch_ws_bytes(int D, int dtype, int ell) {
  SketchPlan p;
  sketch_plan(D, dtype, ell, nullptr, &p);
  return p.bytes;
}

template <typename T, int BF>
static int sketch_t(const T* y, int D, double eps, const int* cap, int ell, uint64_t seed,
                    const TensorDev& out, void* ws, hipStream_t s) {
  SketchPlan p;
  sketch_plan(D, sizeof(T) == 8 ? QTT_F64 : QTT_F32, ell, ws, &p);
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] {
    set_lds_limit((const void*)k_sketch_step<T>, (int)sketch_step_lds(), &attr_err);
  });
  QTT_HIP_CHECK(attr_err);
  StepOut so;
  so.ranks = out.ranks;
  so.status = out.status;
  so.sv = nullptr;
  so.lib_capped = 1;
  so.dbg = nullptr;
  so.delta2 = 0.0;
  T* cores = static_cast<T*>(out.cores);
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  const T* X = y;
  int cur = 0;
  ProbeScope _ps(QTT_K_SKETCH, s);
  for (int k = 1; k <= D - 1; ++k) {
    const long long n = 1LL << (D - k);
    const int mcap = (k == 1) ? 2 : 2 * cap[k - 1];
    // 1. Gram + sketch partials
    const long long nstage = (n + kSkSR - 1) / kSkSR;
    const int blocks = (int)(nstage < kMaxPartials ? nstage : kMaxPartials);
    const size_t lds = sizeof(double) * kSkSR * mcap + sizeof(float) * kSkSR * ell;
    const int kin = k - 1;  // ranks index of r_{k-1}; 0 -> m = 2
    int nparts = blocks;
    if (mcap <= 16 && mcap <= ell) {
      // narrow and exact: the Gram alone, in 2048-value stages
      const long long ns2 = (n * mcap + 2047) / 2048;
      nparts = (int)(ns2 < kMaxPartials ? ns2 : kMaxPartials);
      k_gram_small<T><<<nparts, 256, 0, s>>>(X, n, out.ranks, kin, p.partials, p.pstride);
    } else if (mcap <= 16)
      k_gram_sketch<T, BF, 1><<<blocks, 256, lds, s>>>(X, n, out.ranks, kin, ell, k0, k1, k,
                                                       p.partials, p.pstride);
    else if (mcap <= 32)
      k_gram_sketch<T, BF, 2><<<blocks, 256, lds, s>>>(X, n, out.ranks, kin, ell, k0, k1, k,
                                                       p.partials, p.pstride);
    else if (mcap <= 64)
      k_gram_sketch<T, BF, 4><<<blocks, 256, lds, s>>>(X, n, out.ranks, kin, ell, k0, k1, k,
                                                       p.partials, p.pstride);
    else
      k_gram_sketch<T, BF, 8><<<blocks, 256, lds, s>>>(X, n, out.ranks, kin, ell, k0, k1, k,
                                                       p.partials, p.pstride);
    QTT_LAUNCH_CHECK();
    const int cnt = mcap * mcap + mcap * ell;
    k_sum_partials<<<(cnt + 255) / 256, 256, 0, s>>>(p.partials, p.pstride, nparts, out.ranks,
                                                     kin, ell, p.gy);
    QTT_LAUNCH_CHECK();
    // 2. QR, small eigenproblem, core k
    k_sketch_step<T><<<1, kEigThreads, sketch_step_lds(), s>>>(
        p.gy, k, D, eps, k == 1, ell, p.scal, cap[k], cores, out.off[k - 1], p.umat, p.gT, so);
    QTT_LAUNCH_CHECK();
    // 3. next remainder
    T* Xn = static_cast<T*>(p.xbuf[cur]);
    long long pb = (n * cap[k] + 255) / 256;
    if (pb > 4096) pb = 4096;
    k_sketch_project<T><<<(unsigned)pb, 256, 0, s>>>(X, n, out.ranks, kin, k, p.umat, Xn);
    QTT_LAUNCH_CHECK();
    X = Xn;
    cur ^= 1;
  }
  k_sketch_last<T><<<1, 64, 0, s>>>(X, out.ranks, D, cores, out.off[D - 1], out.ranks);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_round_sketch(int dtype, int bf16, const void* y, int D, double eps, const int* cap,
                     int ell, uint64_t seed, const TensorDev& out, void* ws, hipStream_t s) {
  if (dtype == QTT_F64)
    return bf16 ? sketch_t<double, 1>(static_cast<const double*>(y), D, eps, cap, ell, seed, out,
                                      ws, s)
                : sketch_t<double, 0>(static_cast<const double*>(y), D, eps, cap, ell, seed, out,
                                      ws, s);
  return bf16 ? sketch_t<float, 1>(static_cast<const float*>(y), D, eps, cap, ell, seed, out, ws,
                                   s)
              : sketch_t<float, 0>(static_cast<const float*>(y), D, eps, cap, ell, seed, out, ws,
                                   s);
}

}  // namespace qtt

// TT-SVD and the max-rank TT-RSVD of Section 5 (modifications (1) and (2))
// on a tensor of K modes of size M, FP64, index i = i_1 + M (i_2 + M (...)).
//
// Step k works on the remainder R_k: the unfolding A_k (m x n column-major,
// m = M r_{k-1}, n = M^(K-k)) is stored contiguously, A_k(a, c) = R_k[a + m c].
//   exact step:       one streaming pass forms G = A A^T (fixed-order sum of
//                     per-block partials); the eigensolver gives U (m x r),
//                     r by Algorithm 1's rule and the cap; on a short
//                     unfolding (n <= 64, n < m) one workgroup takes A = Q R
//                     and the eigenproblem of R R^T instead (k_meig);
//   randomised step   (min(M cap_{k-1}, n) > R + p, Algorithms 4 and 5):
//                     Y = A Omega (m x ell, Omega drawn per tile), Q = an
//                     orthonormal basis of range(Y) (eigenvectors of Y^T Y,
//                     one Newton-Schulz polishing step), a second pass forms
//                     G_B = (Q^T A)(Q^T A)^T, its eigenvectors U~ give U = Q U~;
//   both:             R_{k+1} = U^T A (r x n), which is the next unfolding.
// Core k is U read as (r_{k-1}, M, r_k): core[a][i][b] = U[a + r_{k-1} i][b].
// Every streaming pass multiplies on the FP64 matrix cores.
#include <math.h>

#include <mutex>

#include "qtt_eig.hpp"
#include "qtt_internal.hpp"
#include "qtt_philox.hpp"

namespace qtt {

constexpr int kMsMaxEll = 64;        // sketch width limit (ell = R + p)
constexpr int kModesPartials = 512;  // partial results per streaming pass (kMaxM^2 doubles each)
constexpr int kTileElems = 4096;     // doubles of A per tile of the streaming passes
constexpr int kWaveSumElems = 3 * 3 * 256;  // LDS for the cross-wave sum of <= 3 accumulators

typedef double mf64x4 __attribute__((ext_vector_type(4)));

// All streaming passes run on the FP64 matrix cores.  v_mfma_f64_16x16x4f64:
// lane l supplies A entry (row l % 16, k l / 16) and B entry (k l / 16,
// column l % 16); element i of the result is D[4i + l / 16][l % 16].
__device__ __forceinline__ mf64x4 mfma4(double a, double b, mf64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// The tile of columns c0 .. c0 + nc - 1 of A_k is the contiguous block
// R[m c0 .. m (c0 + nc)); it is copied to As[c m + a] as it is.
__device__ __forceinline__ void mload_tile(const double* __restrict__ R, int m, long long c0,
                                           int nc, double* As) {
  const double* src = R + (long long)m * c0;
  const int tot = m * nc;
  if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
    double2* d2 = reinterpret_cast<double2*>(As);
    for (int e = threadIdx.x; e < (tot >> 1); e += 256) d2[e] = s2[e];
    if ((tot & 1) && threadIdx.x == 0) As[tot - 1] = src[tot - 1];
  } else {
    for (int e = threadIdx.x; e < tot; e += 256) As[e] = src[e];
  }
}

// Register staging of the next tile (NP double2 per thread, so tiles of
// <= 512 NP doubles): its loads are issued before the current tile's
// products and land in LDS after them.  Needs R + m c0 16-byte aligned for
// every tile (R aligned, tc even).
template <int NP = kTileElems / 512>
struct TileStage {
  double2 v[NP];
  int tot;
  __device__ __forceinline__ void load(const double* __restrict__ R, int m, long long c0,
                                       int nc) {
    const double2* s2 = reinterpret_cast<const double2*>(R + (long long)m * c0);
    tot = m * nc;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int e = threadIdx.x + 256 * p;
      v[p] = e < (tot >> 1) ? s2[e] : make_double2(0.0, 0.0);
    }
  }
  __device__ __forceinline__ void store(const double* __restrict__ R, int m, long long c0,
                                        double* As) const {
    double2* d2 = reinterpret_cast<double2*>(As);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int e = threadIdx.x + 256 * p;
      if (e < (tot >> 1)) d2[e] = v[p];
    }
    if ((tot & 1) && threadIdx.x == 0) As[tot - 1] = R[(long long)m * c0 + tot - 1];
  }
};

// Tile t of the grid-stride loop into As: from the registers staged during
// the previous tile when aligned (then the next tile is staged), else loaded
// directly.
template <int NP>
__device__ __forceinline__ void next_tile(const double* __restrict__ R, int m, long long n,
                                          int tc, long long t, bool aligned, TileStage<NP>& st,
                                          double* As) {
  const long long c0 = t * tc;
  const int nc = (int)((n - c0) < tc ? (n - c0) : tc);
  if (aligned) {
    st.store(R, m, c0, As);
    const long long tn = t + gridDim.x;
    if (tn * tc < n) {
      const long long cn0 = tn * tc;
      st.load(R, m, cn0, (int)((n - cn0) < tc ? (n - cn0) : tc));
    }
  } else {
    mload_tile(R, m, c0, nc, As);
  }
}

__device__ __forceinline__ bool stage_ok(const double* R, int m, int tc,
                                         int cap = kTileElems) {
  return (reinterpret_cast<uintptr_t>(R) & 15) == 0 && (tc & 1) == 0 &&
         (long long)m * tc <= cap;
}

// Upper-triangle block idx (< nb (nb + 1) / 2) of an nb x nb block grid, in
// the order (0,0), (0,1), ..., (0,nb-1), (1,1), ...
__device__ __forceinline__ void tri_block(int idx, int nb, int& bi, int& bj) {
  int a = 0;
  while (a < nb && idx >= nb - a) {
    idx -= nb - a;
    ++a;
  }
  bi = a;
  bj = a + idx;
}

// G += T T^T for the column groups gr = g0, g0 + gs, ... (4 columns each) of
// the LDS tile T (column c at T + c ldt, rows < m, nc columns): accumulator t
// holds the 16 x 16 block (bi[t], bj[t]) when on[t].
template <int NA>
__device__ __forceinline__ void mfma_gram_tile(const double* T, int ldt, int m, int nc,
                                               const int* bi, const int* bj, const bool* on,
                                               int g0, int gs, mf64x4* g) {
  const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
  const int ng = (nc + 3) >> 2;
  for (int gr = g0; gr < ng; gr += gs) {
    const int c = 4 * gr + lk;
    const bool cin = c < nc;
#pragma unroll
    for (int t = 0; t < NA; ++t) {
      if (!on[t]) continue;  // wave-uniform
      const int ra = 16 * bi[t] + lr, rb = 16 * bj[t] + lr;
      const double x = (cin && ra < m) ? T[c * ldt + ra] : 0.0;
      const double y = (cin && rb < m) ? T[c * ldt + rb] : 0.0;
      g[t] = mfma4(x, y, g[t]);
    }
  }
}

// Waves 1..3 hand their first na (<= 3) accumulators to wave 0 through LDS
// (buf: kWaveSumElems doubles); wave 0 adds them in wave order.  Every thread
// of the block calls it.
template <int NA>
__device__ __forceinline__ void mfma_wave_sum(double* buf, int na, mf64x4* g) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (w > 0) {
#pragma unroll
    for (int t = 0; t < NA; ++t)
      if (t < na && t < 3)
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[(((w - 1) * 3 + t) * 4 + i) * 64 + l] = g[t][i];
  }
  __syncthreads();
  if (w == 0) {
    for (int ww = 1; ww < 4; ++ww)
#pragma unroll
      for (int t = 0; t < NA; ++t)
        if (t < na && t < 3)
#pragma unroll
          for (int i = 0; i < 4; ++i) g[t][i] += buf[(((ww - 1) * 3 + t) * 4 + i) * 64 + l];
  }
}

// Symmetric partial Gram (m x m, row-major) from the upper-triangle blocks.
template <int NA>
__device__ __forceinline__ void mfma_gram_store(double* P, int m, const int* bi, const int* bj,
                                                const bool* on, const mf64x4* g) {
  const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
#pragma unroll
  for (int t = 0; t < NA; ++t) {
    if (!on[t]) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * bi[t] + 4 * i + lk, col = 16 * bj[t] + lr;
      if (row < m && col < m) {
        P[row * m + col] = g[t][i];
        if (bi[t] != bj[t]) P[col * m + row] = g[t][i];
      }
    }
  }
}

// ------------------------------------------------------------- Gram pass
// Partial G = A A^T over this block's column tiles (grid-stride), m <= 16 MB.
// With at least 4 upper-triangle blocks the waves split the blocks, else the
// column groups (and are summed at the end).
template <int MB>
__global__ void __launch_bounds__(256) k_mgram(const double* __restrict__ R, int M,
                                               const int32_t* __restrict__ ranks, int k,
                                               long long n, int tc, double* __restrict__ partials,
                                               int pstride) {
  constexpr int NB = MB * (MB + 1) / 2;
  constexpr bool SPLIT = NB >= 4;
  constexpr int NA = SPLIT ? (NB + 3) / 4 : NB;
  extern __shared__ double As[];  // tc x m, at least kWaveSumElems
  const int m = M * ranks[k - 1];
  const int w = threadIdx.x >> 6;
  int bi[NA], bj[NA];
  bool on[NA];
  mf64x4 g[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) {
    const int idx = SPLIT ? w + 4 * t : t;
    on[t] = idx < NB;
    bi[t] = 0;
    bj[t] = 0;
    if (on[t]) tri_block(idx, MB, bi[t], bj[t]);
    g[t] = mf64x4{0.0, 0.0, 0.0, 0.0};
  }
  const long long ntile = (n + tc - 1) / tc;
  const bool aligned = stage_ok(R, m, tc);
  TileStage<> st;
  if (aligned && blockIdx.x < ntile) {
    const long long c0 = (long long)blockIdx.x * tc;
    st.load(R, m, c0, (int)((n - c0) < tc ? (n - c0) : tc));
  }
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * tc;
    const int nc = (int)((n - c0) < tc ? (n - c0) : tc);
    __syncthreads();
    next_tile(R, m, n, tc, t, aligned, st, As);
    __syncthreads();
    mfma_gram_tile<NA>(As, m, m, nc, bi, bj, on, SPLIT ? 0 : w, SPLIT ? 1 : 4, g);
  }
  if (!SPLIT) {
    mfma_wave_sum<NA>(As, NB, g);
    if (w != 0) return;
  }
  mfma_gram_store<NA>(partials + (size_t)blockIdx.x * pstride, m, bi, bj, on, g);
}

// ----------------------------------------------------------- sketch pass
// Partial Y = A Omega (m x ell, row-major) over this block's column tiles;
// Omega[c][j] = omega_entry(c, j, k, seed) for the global column c, drawn
// into LDS per tile (Om: tc x EL, EL = ell rounded up to 16, zero padded).
template <int MB>
__global__ void __launch_bounds__(256) k_msketch(const double* __restrict__ R, int M,
                                                 const int32_t* __restrict__ ranks, int k,
                                                 long long n, int tc, int as_cap, int ell,
                                                 uint32_t s0, uint32_t s1,
                                                 double* __restrict__ partials, int pstride) {
  constexpr int NA = MB < 3 ? 3 : MB;
  extern __shared__ double As[];  // tc x m (as_cap doubles), then Om
  const int m = M * ranks[k - 1];
  const int EB = (ell + 15) >> 4, EL = 16 * EB;
  double* Om = As + as_cap;
  const int NB = MB * EB;
  const bool split = NB >= 4;  // block-uniform
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  int bi[NA], bj[NA];
  bool on[NA];
  mf64x4 g[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) {
    const int idx = split ? w + 4 * t : t;
    on[t] = idx < NB;
    bi[t] = on[t] ? idx / EB : 0;
    bj[t] = on[t] ? idx - (idx / EB) * EB : 0;
    g[t] = mf64x4{0.0, 0.0, 0.0, 0.0};
  }
  // the padding columns ell .. EL - 1 of Om stay zero
  for (int e = tid; e < tc * EL; e += 256) Om[e] = 0.0;
  const long long ntile = (n + tc - 1) / tc;
  const bool aligned = stage_ok(R, m, tc);
  TileStage<> st;
  if (aligned && blockIdx.x < ntile) {
    const long long c0 = (long long)blockIdx.x * tc;
    st.load(R, m, c0, (int)((n - c0) < tc ? (n - c0) : tc));
  }
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * tc;
    const int nc = (int)((n - c0) < tc ? (n - c0) : tc);
    __syncthreads();
    next_tile(R, m, n, tc, t, aligned, st, As);
    for (int e = tid; e < tc * ell; e += 256) {
      const int c = e / ell, j = e - c * ell;
      Om[c * EL + j] = c < nc ? omega_entry(c0 + c, j, k, s0, s1) : 0.0;
    }
    __syncthreads();
    const int ng = (nc + 3) >> 2;
    for (int gr = split ? 0 : w; gr < ng; gr += split ? 1 : 4) {
      const int c = 4 * gr + lk;
      const bool cin = c < nc;
#pragma unroll
      for (int u = 0; u < NA; ++u) {
        if (!on[u]) continue;
        const int ra = 16 * bi[u] + lr;
        const double x = (cin && ra < m) ? As[c * m + ra] : 0.0;
        const double y = Om[c * EL + 16 * bj[u] + lr];
        g[u] = mfma4(x, y, g[u]);
      }
    }
  }
  if (!split) {
    mfma_wave_sum<NA>(As, NB, g);
    if (w != 0) return;
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    if (!on[u]) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int a = 16 * bi[u] + 4 * i + lk, j = 16 * bj[u] + lr;
      if (a < m && j < ell) P[a * ell + j] = g[u][i];
    }
  }
}

// Y^T = A^T W for a tile (W: m x q row-major in LDS): work items (column
// block cb, basis block qb) round-robin over the waves, the k loop over the
// m rows of A.  Result entry (tile column c, basis vector j) goes to
// put(c, j, value) for j < q (tile columns >= nc come out zero).
template <class Put>
__device__ __forceinline__ void mfma_tile_times(const double* As, int m, int nc, int tc,
                                                const double* Ws, int q, Put put) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
  const int QB = (q + 15) >> 4, items = (tc >> 4) * QB;
  for (int it = w; it < items; it += 4) {
    const int cb = it / QB, qb = it - cb * QB;
    const int c = 16 * cb + lr, j = 16 * qb + lr;
    const bool cin = c < nc, jin = j < q;
    // four k steps per batch: their operands are read first, then the
    // products go to two accumulators in turn
    mf64x4 acc = mf64x4{0.0, 0.0, 0.0, 0.0}, acc1 = acc;
    for (int a0 = 0; a0 < m; a0 += 16) {
      double x[4], y[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int a = a0 + 4 * u + lk;
        const bool ain = a < m;
        x[u] = (ain && cin) ? As[c * m + a] : 0.0;
        y[u] = (ain && jin) ? Ws[a * q + j] : 0.0;
      }
      acc = mfma4(x[0], y[0], acc);
      acc1 = mfma4(x[1], y[1], acc1);
      acc = mfma4(x[2], y[2], acc);
      acc1 = mfma4(x[3], y[3], acc1);
    }
    acc += acc1;
    if (jin) {
#pragma unroll
      for (int i = 0; i < 4; ++i) put(16 * cb + 4 * i + lk, j, acc[i]);
    }
  }
}

// ---------------------------------------------------- G_B = (Q^T A)(Q^T A)^T
// Q: m x q row-major (q = iq[0] <= ell).  Per tile B = Q^T A (q x tc) goes to
// LDS (column c at Bs + c q), then the partial q x q Gram of its columns.
__global__ void __launch_bounds__(256) k_mbgram(const double* __restrict__ R, int M,
                                                const int32_t* __restrict__ ranks, int k,
                                                long long n, int tc, int as_cap, int mcap,
                                                int ell, const double* __restrict__ Q,
                                                const int32_t* __restrict__ iq,
                                                double* __restrict__ partials, int pstride) {
  constexpr int NA = 3;
  extern __shared__ double sm[];
  const int m = M * ranks[k - 1];
  const int q = iq[0];
  double* As = sm;                     // tc x m (as_cap doubles)
  double* Qs = As + as_cap;            // m x q
  double* Bs = Qs + mcap * ell;        // tc x q
  const int tid = threadIdx.x, w = tid >> 6;
  for (int e = tid; e < m * q; e += 256) Qs[e] = Q[e];
  const int QB = (q + 15) >> 4;
  const int NB = QB * (QB + 1) / 2;  // <= 10
  const bool split = NB >= 4;
  int bi[NA], bj[NA];
  bool on[NA];
  mf64x4 g[NA];
#pragma unroll
  for (int t = 0; t < NA; ++t) {
    const int idx = split ? w + 4 * t : t;
    on[t] = idx < NB;
    bi[t] = 0;
    bj[t] = 0;
    if (on[t]) tri_block(idx, QB, bi[t], bj[t]);
    g[t] = mf64x4{0.0, 0.0, 0.0, 0.0};
  }
  const long long ntile = (n + tc - 1) / tc;
  const bool aligned = stage_ok(R, m, tc);
  TileStage<> st;
  if (aligned && blockIdx.x < ntile) {
    const long long c0 = (long long)blockIdx.x * tc;
    st.load(R, m, c0, (int)((n - c0) < tc ? (n - c0) : tc));
  }
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * tc;
    const int nc = (int)((n - c0) < tc ? (n - c0) : tc);
    __syncthreads();
    next_tile(R, m, n, tc, t, aligned, st, As);
    __syncthreads();
    mfma_tile_times(As, m, nc, tc, Qs, q, [&](int c, int j, double v) { Bs[c * q + j] = v; });
    __syncthreads();
    mfma_gram_tile<NA>(Bs, q, q, nc, bi, bj, on, split ? 0 : w, split ? 1 : 4, g);
  }
  if (!split) {
    mfma_wave_sum<NA>(As, NB, g);
    if (w != 0) return;
  }
  mfma_gram_store<NA>(partials + (size_t)blockIdx.x * pstride, q, bi, bj, on, g);
}

// -------------------------------------------------------- eigen problems
struct MEig {
  double *A, *V, *lam, *sx;
  int *perm, *iscr;
  int lda;
};

__device__ __forceinline__ MEig meig_layout(double* smem, int E, double* gV) {
  MEig L;
  if (E <= kEigLds) {
    L.lda = kEigLds + 1;
    L.A = smem;
    L.V = L.A + L.lda * L.lda;
    L.lam = L.V + L.lda * L.lda;
  } else {
    // orders 65..128: the matrix in LDS, the eigenvectors in global memory
    L.lda = kMaxM + 1;
    L.A = smem;
    L.V = gV;
    L.lam = L.A + L.lda * L.lda;
  }
  L.sx = L.lam + kMaxM + 8;
  L.perm = (int*)(L.sx + kEigScratch);
  L.iscr = L.perm + kMaxM + 8;
  return L;
}

// status (may be null) receives QTT_STATUS_NONFINITE for a non-finite matrix
// and, when lib_capped, QTT_STATUS_RANKCAP for an eps-rank above cap
template <class MP, class MPV>
__device__ int meig_solve(const MEig& L, MP A, MPV V, int E, double tau2, int cap, int32_t* rk,
                          int k, int32_t* status = nullptr, int lib_capped = 0) {
  StepOut so;
  so.ranks = rk;
  so.status = status;
  so.sv = nullptr;
  so.lib_capped = lib_capped;
  so.dbg = nullptr;
  so.delta2 = 0.0;
  return solve_and_truncate<kEigThreads, true>(A, V, E, L.lda, lds(L.sx), lds(L.iscr), lds(L.lam),
                                              lds(L.perm), tau2, cap, k, so);
}

// Step k's truncated eigendecomposition.  Writes ranks[k], core k and U
// (m x r, row-major) to umat.
//   use_q = 0, exact step:      G is m x m and U = V[:, :r];
//   use_q = 1, randomised step: G is G_B (q x q) and U = Q V[:, :r];
//   use_q = 2, exact step on a short unfolding (Q = A_k itself, n = ncol
//   columns, n <= 64): for m > n, A = Q_A R_A by Gram-Schmidt (applied
//   twice) in LDS, G = R_A R_A^T (n x n, the same nonzero eigenvalues as
//   A A^T) and U = Q_A V[:, :r]; for m <= n, G = A A^T formed here.
__global__ void __launch_bounds__(kEigThreads) k_meig(const double* G, int M, int32_t* ranks,
                                                      int k, int use_q, const double* Q,
                                                      const int32_t* iq, double* scal,
                                                      int cap_k, double* cores, long long off_k,
                                                      double* umat, double* gV,
                                                      int set_tau, double eps, int K, int ncol,
                                                      int32_t* status, int lib_capped) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int rp = ranks[k - 1];
  const int m = M * rp;
  const bool tall = use_q == 2 && m > ncol;  // uniform
  const int q = use_q == 1 ? iq[0] : (tall ? ncol : m);
  const int E = q;
  const MEig L = meig_layout(smem, E, gV);
  const double* Qsrc = Q;  // the basis U is taken in (use_q != 0)
  if (use_q == 2) {
    const int n = ncol;
    const double* A = Q;  // A(a, c) = A[a + m c]
    if (!tall) {
      for (int e = tid; e < m * m; e += kEigThreads) {
        const int a = e / m, b = e - a * m;
        double t = 0.0;
        for (int c = 0; c < n; ++c) t = fma(A[a + m * c], A[b + m * c], t);
        L.A[a * L.lda + b] = t;
      }
    } else {
      // Q_A (m x n, row-major) after the solver's arrays
      double* Qa = reinterpret_cast<double*>(L.iscr + 8 + 256);
      ldsd cn = lds(L.sx), al = lds(L.sx + 64), fr = lds(L.sx + 128);
      for (int e = tid; e < m * n; e += kEigThreads) {
        const int c = e / m, a = e - c * m;
        Qa[a * n + c] = A[e];
      }
      __syncthreads();
      if (tid < 64) {
        double t = 0.0;
        for (int e = tid; e < m * n; e += 64) t = fma(Qa[e], Qa[e], t);
        t = sum64(t);
        if (tid == 0) fr[0] = t;
      }
      __syncthreads();
      const double fro2 = fr[0];
      for (int j = 0; j < n; ++j) {
        cgs2_col<kEigThreads>(lds(Qa), m, n, j, cn, al);
        double t = col_norm2(lds(Qa), m, n, j);
        if (!(t > 1e-28 * fro2)) {
          // (numerically) dependent column: any unit vector orthogonal to
          // the earlier ones; a dense deterministic start (an integer hash
          // of (i, j)) has a component outside their span (j < n < m)
          __syncthreads();
          for (int i = tid; i < m; i += kEigThreads) {
            const unsigned int h =
                (unsigned int)(i + 1) * 2654435761u ^ (unsigned int)(j + 7) * 40503u;
            Qa[i * n + j] = (double)(h >> 8) * (1.0 / 8388608.0) - 1.0;
          }
          __syncthreads();
          cgs2_col<kEigThreads>(lds(Qa), m, n, j, cn, al);
          t = col_norm2(lds(Qa), m, n, j);
        }
        const double inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
        __syncthreads();
        for (int i = tid; i < m; i += kEigThreads) Qa[i * n + j] *= inv;
        if (tid == 0) cn[j] = 1.0;
        __syncthreads();
      }
      // R_A = Q_A^T A (in V), then G = R_A R_A^T
      for (int e = tid; e < n * n; e += kEigThreads) {
        const int c = e / n, c2 = e - c * n;
        double t = 0.0;
        for (int a = 0; a < m; ++a) t = fma(Qa[a * n + c], A[a + m * c2], t);
        L.V[c * L.lda + c2] = t;
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += kEigThreads) {
        const int i = e / n, j = e - i * n;
        double t = 0.0;
        for (int c = 0; c < n; ++c) t = fma(L.V[i * L.lda + c], L.V[j * L.lda + c], t);
        L.A[i * L.lda + j] = t;
      }
      Qsrc = Qa;
    }
  } else {
    for (int e = tid; e < E * E; e += kEigThreads) {
      const int a = e / E, b = e - a * E;
      L.A[a * L.lda + b] = G[e];
    }
    if (set_tau && tid == 0) {
      // exact first step: ||x||^2 is the trace of its Gram
      double tr = 0.0;
      for (int a = 0; a < E; ++a) tr += G[a * E + a];
      scal[0] = tr;
      scal[1] = (K > 1) ? eps * eps * tr / (double)(K - 1) : 0.0;
    }
  }
  __syncthreads();
  int r;
  if (E <= kEigLds)
    r = meig_solve(L, lds(L.A), lds(L.V), E, scal[1], cap_k, ranks, k, status, lib_capped);
  else
    r = meig_solve(L, lds(L.A), L.V, E, scal[1], cap_k, ranks, k, status, lib_capped);
  // U (m x r) and core k
  const bool basis = use_q == 1 || tall;
  for (int e = tid; e < m * r; e += kEigThreads) {
    const int b = e % r, t = e / r;
    const int i = t % M, ai = t / M;   // core order (r_{k-1}, M, r_k)
    const int row = ai + rp * i;       // unfolding row of that entry
    const int col = L.perm[b];
    double u;
    if (basis) {
      u = 0.0;
      for (int c = 0; c < q; ++c) u = fma(Qsrc[row * q + c], L.V[c * L.lda + col], u);
    } else {
      u = L.V[row * L.lda + col];
    }
    cores[off_k + e] = u;
    umat[row * r + b] = u;
  }
}

// Orthonormal basis of range(Y) (Y: m x ell, row-major): eigenvectors W of
// C = Y^T Y with eigenvalues above 1e-24 of the largest, Q1 = Y W L^-1/2,
// then Q = Q1 (3I - Q1^T Q1) / 2.  Writes Q (m x q, row-major) and iq[0] = q.
// Y, and later Q1, are read from LDS (after the solver's arrays); Q1 passes
// through global memory once, since it is formed from Y in place.
__global__ void __launch_bounds__(kEigThreads) k_mqr(const double* Y, int M, const int32_t* ranks,
                                                     int k, int ell, double* Q1, double* Q,
                                                     int32_t* iq) {
  extern __shared__ double smem[];
  __shared__ int32_t rk[4];
  const int tid = threadIdx.x;
  const int m = M * ranks[k - 1];
  const int E = ell;  // <= 64: LDS
  const MEig L = meig_layout(smem, E, nullptr);
  double* Ys = reinterpret_cast<double*>(L.iscr + 8 + 256);  // <= kMaxM x kMsMaxEll
  for (int e = tid; e < m * ell; e += kEigThreads) Ys[e] = Y[e];
  __syncthreads();
  for (int e = tid; e < E * E; e += kEigThreads) {
    const int a = e / E, b = e - a * E;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(Ys[i * ell + a], Ys[i * ell + b], s);
    L.A[a * L.lda + b] = s;
  }
  __syncthreads();
  // all eigenpairs (tolerance 0, no cap below ell)
  const int r = meig_solve(L, lds(L.A), lds(L.V), E, 0.0, E, rk, 1);
  const double l0 = L.lam[0];
  int qn = 0;
  for (int b = 0; b < r; ++b) qn += (L.lam[b] > 1e-24 * l0) ? 1 : 0;
  if (!(l0 > 0.0)) {
    // Y = 0 (a zero unfolding): any unit vector spans what is needed
    qn = 1;
    for (int i = tid; i < m; i += kEigThreads) Q1[i] = (i == 0) ? 1.0 : 0.0;
  } else {
    // Q1 = Y W L^-1/2
    for (int e = tid; e < m * qn; e += kEigThreads) {
      const int i = e / qn, b = e - i * qn;
      double s = 0.0;
      for (int c = 0; c < ell; ++c) s = fma(Ys[i * ell + c], L.V[c * L.lda + L.perm[b]], s);
      Q1[e] = s / sqrt(L.lam[b]);
    }
  }
  __syncthreads();
  for (int e = tid; e < m * qn; e += kEigThreads) Ys[e] = Q1[e];
  __syncthreads();
  // S = (3I - Q1^T Q1) / 2 in the matrix area (free after the solve)
  double* Sq = L.A;
  for (int e = tid; e < qn * qn; e += kEigThreads) {
    const int a = e / qn, b = e - a * qn;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(Ys[i * qn + a], Ys[i * qn + b], s);
    Sq[e] = (a == b ? 1.5 : 0.0) - 0.5 * s;
  }
  __syncthreads();
  for (int e = tid; e < m * qn; e += kEigThreads) {
    const int i = e / qn, b = e - i * qn;
    double s = 0.0;
    for (int c = 0; c < qn; ++c) s = fma(Ys[i * qn + c], Sq[c * qn + b], s);
    Q[e] = s;
  }
  if (tid == 0) iq[0] = qn;
}

// ------------------------------------------------------------ projection
// R_{k+1}[b + r c] = sum_a U[a][b] A(a, c): U (m x r, row-major) in LDS
// after the tile (as_cap doubles).
__global__ void __launch_bounds__(256) k_mproj(const double* __restrict__ R, int M,
                                               const int32_t* __restrict__ ranks, int k,
                                               long long n, int tc, int as_cap,
                                               const double* __restrict__ U,
                                               double* __restrict__ Rn) {
  extern __shared__ double sm[];
  const int m = M * ranks[k - 1];
  const int r = ranks[k];
  double* As = sm;
  double* Us = sm + as_cap;
  for (int e = threadIdx.x; e < m * r; e += 256) Us[e] = U[e];
  const long long ntile = (n + tc - 1) / tc;
  constexpr int NP = 2 * kTileElems / 512;  // tiles up to 2 kTileElems doubles
  const bool aligned = stage_ok(R, m, tc, 2 * kTileElems);
  TileStage<NP> st;
  if (aligned && blockIdx.x < ntile) {
    const long long c0 = (long long)blockIdx.x * tc;
    st.load(R, m, c0, (int)((n - c0) < tc ? (n - c0) : tc));
  }
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * tc;
    const int nc = (int)((n - c0) < tc ? (n - c0) : tc);
    __syncthreads();
    next_tile(R, m, n, tc, t, aligned, st, As);
    __syncthreads();
    double* dst = Rn + (long long)r * c0;
    mfma_tile_times(As, m, nc, tc, Us, r, [&](int c, int b, double v) {
      if (c < nc) dst[(long long)r * c + b] = v;
    });
  }
}

// ------------------------------------------------------------ bookkeeping
__global__ void k_mstart(double* scal, double eps, int K, int32_t* ranks, int have_norm) {
  if (threadIdx.x == 0) {
    if (have_norm) scal[1] = (K > 1) ? eps * eps * scal[0] / (double)(K - 1) : 0.0;
    ranks[0] = 1;
    ranks[K] = 1;
  }
}

// last core (r_{K-1}, M, 1) from the remainder (r x M column-major)
__global__ void k_mlast(const double* R, int M, const int32_t* ranks, int K, double* core) {
  const int r = ranks[K - 1];
  for (int e = threadIdx.x + blockIdx.x * blockDim.x; e < r * M; e += blockDim.x * gridDim.x) {
    const int a = e / M, i = e - a * M;
    core[e] = R[a + r * i];
  }
}

// ==================================================================== host
int modes_caps(int K, int M, int max_rank, int32_t* cap) {
  int R = max_rank > 0 ? max_rank : kMaxRank;
  if (R > kMaxRank) R = kMaxRank;
  if (R * M > kMaxM) R = kMaxM / M;
  for (int k = 0; k <= K; ++k) {
    // min(M^k, M^(K-k), R) without overflow
    long long lo = 1, hi = 1;
    for (int j = 0; j < k && lo < R; ++j) lo *= M;
    for (int j = 0; j < K - k && hi < R; ++j) hi *= M;
    long long c = R;
    if (lo < c) c = lo;
    if (hi < c) c = hi;
    cap[k] = (k == 0 || k == K) ? 1 : (int)c;
  }
  return R;
}

struct ModesPlan {
  double *scal, *dotp, *partials, *gram, *gramb, *y, *umat, *q1, *q, *gV, *rbuf[2];
  int32_t* iq;
  int pstride;
  size_t bytes;
};

static ModesPlan modes_plan(void* ws, int K, int M) {
  long long N = 1;
  for (int k = 0; k < K; ++k) N *= M;
  Arena ar(ws);
  ModesPlan p;
  p.pstride = kMaxM * kMaxM;
  p.scal = ar.take<double>(16);
  p.dotp = ar.take<double>(kDotPartials);
  p.iq = ar.take<int32_t>(16);
  p.partials = ar.take<double>((size_t)kModesPartials * p.pstride);
  p.gram = ar.take<double>((size_t)kMaxM * kMaxM);
  p.gramb = ar.take<double>((size_t)kMsMaxEll * kMsMaxEll);
  p.y = ar.take<double>((size_t)kMaxM * kMsMaxEll);
  p.umat = ar.take<double>((size_t)kMaxM * kMaxRank);
  p.q1 = ar.take<double>((size_t)kMaxM * kMsMaxEll);
  p.q = ar.take<double>((size_t)kMaxM * kMsMaxEll);
  p.gV = ar.take<double>((size_t)(kMaxM + 1) * (kMaxM + 1));
  p.rbuf[0] = ar.take<double>((size_t)N);
  p.rbuf[1] = ar.take<double>((size_t)N);
  p.bytes = ar.size();
  return p;
}

size_t modes_ws_bytes(int K, int M, int method, int oversample) {
  (void)method;
  (void)oversample;
  return modes_plan(nullptr, K, M).bytes;
}

// LDS of the eigen kernels: two matrices of order <= 64, or one of order
// <= 128 (k_meig only), plus the solver's vectors
static size_t lds_meig_small() {
  const int lda = kEigLds + 1;
  return sizeof(double) * (2 * lda * lda + (kMaxM + 8) + kEigScratch) +
         sizeof(int) * (kMaxM + 8 + 8 + 256);
}
static size_t lds_mqr() { return lds_meig_small() + sizeof(double) * kMaxM * kMsMaxEll; }
static size_t lds_meig() {
  const int lda = kMaxM + 1;
  const size_t big = sizeof(double) * (lda * lda + (kMaxM + 8) + kEigScratch) +
                     sizeof(int) * (kMaxM + 8 + 8 + 256);
  // the short-unfolding step keeps Q_A (<= kMaxM x kEigLds) after the small layout
  const size_t tall = lds_meig_small() + sizeof(double) * kMaxM * kEigLds;
  return big > tall ? big : tall;
}

// Columns per tile: about kTileElems doubles of A, a multiple of 16 in
// [lo, hi].
static int mtile(int mcap, int lo, int hi) {
  int tc = (kTileElems / mcap) & ~15;
  return tc < lo ? lo : (tc > hi ? hi : tc);
}
static int as_elems(int tc, int mcap) {
  return tc * mcap > kWaveSumElems ? tc * mcap : kWaveSumElems;
}

constexpr int kMaxStreamLds = 150 * 1024;

template <int MB>
static void set_stream_attrs(hipError_t* e) {
  set_lds_limit((const void*)k_mgram<MB>, kMaxStreamLds, e);
  set_lds_limit((const void*)k_msketch<MB>, kMaxStreamLds, e);
}

template <int MB>
static void launch_stream_mb(int which, const double* R, int M, const int32_t* ranks, int k,
                             long long n, int blocks, int tc, int as_cap, int ell, uint64_t seed,
                             double* partials, int pstride, size_t lds, hipStream_t s) {
  if (which == 0)
    k_mgram<MB><<<blocks, 256, lds, s>>>(R, M, ranks, k, n, tc, partials, pstride);
  else
    k_msketch<MB><<<blocks, 256, lds, s>>>(R, M, ranks, k, n, tc, as_cap, ell,
                                           (uint32_t)(seed & 0xFFFFFFFFu),
                                           (uint32_t)(seed >> 32), partials, pstride);
}

// One streaming pass over A_k: 0 = Gram (m x m partials), 1 = sketch
// (m x ell), 2 = G_B (ell x ell at most).  Sets the number of partials and
// their stride for the fixed-order reduction.
static int stream_pass(int which, const double* R, int M, int mcap, int32_t* ranks, int k,
                       long long n, int* nparts, int* pstride, int ell, uint64_t seed,
                       const ModesPlan& P, hipStream_t s) {
  const long long sz = which == 0 ? (long long)mcap * mcap
                                  : (which == 1 ? (long long)mcap * ell : (long long)ell * ell);
  int tc, as_cap;
  size_t lds;
  if (which == 0) {
    tc = mtile(mcap, 16, 1024);
    as_cap = as_elems(tc, mcap);
    lds = sizeof(double) * (size_t)as_cap;
  } else if (which == 1) {
    tc = mtile(mcap, 16, 256);
    as_cap = as_elems(tc, mcap);
    lds = sizeof(double) * ((size_t)as_cap + (size_t)tc * (16 * ((ell + 15) / 16)));
  } else {
    tc = mtile(mcap, 32, 512);
    as_cap = as_elems(tc, mcap);
    lds = sizeof(double) * ((size_t)as_cap + (size_t)mcap * ell + (size_t)tc * ell);
  }
  if (lds > (size_t)kMaxStreamLds) return QTT_EINVAL;
  const long long ntile = (n + tc - 1) / tc;
  const long long cap_parts = (long long)kModesPartials * P.pstride / sz;
  long long b = ntile < 1024 ? ntile : 1024;
  if (b > cap_parts) b = cap_parts;
  const int blocks = (int)(b < 1 ? 1 : b);
  *nparts = blocks;
  *pstride = (int)sz;
  if (which == 2) {
    k_mbgram<<<blocks, 256, lds, s>>>(R, M, ranks, k, n, tc, as_cap, mcap, ell, P.q, P.iq,
                                      P.partials, (int)sz);
  } else {
    const int mb = (mcap + 15) / 16;
    switch (mb) {
#define QTT_MB_CASE(X)                                                                         \
  case X:                                                                                      \
    launch_stream_mb<X>(which, R, M, ranks, k, n, blocks, tc, as_cap, ell, seed, P.partials,   \
                        (int)sz, lds, s);                                                      \
    break;
      QTT_MB_CASE(1)
      QTT_MB_CASE(2)
      QTT_MB_CASE(3)
      QTT_MB_CASE(4)
      QTT_MB_CASE(5)
      QTT_MB_CASE(6)
      QTT_MB_CASE(7)
      QTT_MB_CASE(8)
#undef QTT_MB_CASE
      default: return QTT_EINVAL;
    }
  }
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_decompose_modes(const double* x, int K, int M, double eps, int method, int oversample,
                        uint64_t seed, const int32_t* cap, int32_t* ranks, double* cores,
                        int32_t* status, int lib_capped, void* ws, hipStream_t s) {
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] {
    hipError_t* e = &attr_err;
    set_lds_limit((const void*)k_meig, (int)lds_meig(), e);
    set_lds_limit((const void*)k_mqr, (int)lds_mqr(), e);
    set_lds_limit((const void*)k_mproj, kMaxStreamLds, e);
    set_lds_limit((const void*)k_mbgram, kMaxStreamLds, e);
    set_stream_attrs<1>(e);
    set_stream_attrs<2>(e);
    set_stream_attrs<3>(e);
    set_stream_attrs<4>(e);
    set_stream_attrs<5>(e);
    set_stream_attrs<6>(e);
    set_stream_attrs<7>(e);
    set_stream_attrs<8>(e);
  });
  QTT_HIP_CHECK(attr_err);
  const ModesPlan P = modes_plan(ws, K, M);
  long long N = 1;
  for (int k = 0; k < K; ++k) N *= M;
  int Rmax = 0;
  for (int k = 1; k <= K; ++k)
    if (cap[k] > Rmax) Rmax = cap[k];
  const int ell0 = (method == 1) ? Rmax + oversample : 0;
  // ||x||^2: the trace of the first step's Gram when that step is exact,
  // else one dot pass
  const bool first_exact = !(method == 1 && ((long long)M < N / M ? (long long)M : N / M) > ell0);
  int rc = QTT_OK;
  if (!first_exact || K == 1) {
    rc = run_dot(QTT_F64, x, x, N, P.dotp, P.scal, s);
    if (rc) return rc;
  }
  k_mstart<<<1, 64, 0, s>>>(P.scal, eps, K, ranks, (!first_exact || K == 1) ? 1 : 0);
  QTT_LAUNCH_CHECK();
  long long off = 0;
  const double* cur = x;
  int bi = 0;
  long long n = N;
  const int ell = ell0;
  for (int k = 1; k < K; ++k) {
    n /= M;  // columns of A_k
    const int mcap = M * cap[k - 1];
    const bool rs = (method == 1) && ((long long)mcap < n ? (long long)mcap : n) > ell;
    int np = 0, ps = 0;
    // an exact step on an unfolding with few columns works from A_k itself
    const bool short_unf = !rs && k > 1 && n <= kEigLds && n < mcap;
    if (short_unf) {
      k_meig<<<1, kEigThreads, lds_meig(), s>>>(nullptr, M, ranks, k, 2, cur, P.iq, P.scal,
                                                cap[k], cores, off, P.umat, P.gV, 0, eps, K,
                                                (int)n, status, lib_capped);
      QTT_LAUNCH_CHECK();
    } else if (!rs) {
      rc = stream_pass(0, cur, M, mcap, ranks, k, n, &np, &ps, 0, seed, P, s);
      if (rc) return rc;
      rc = launch_reduce(P.partials, ps, np, mcap * mcap, P.gram, s);
      if (rc) return rc;
      k_meig<<<1, kEigThreads, lds_meig(), s>>>(P.gram, M, ranks, k, 0, nullptr, P.iq, P.scal,
                                                cap[k], cores, off, P.umat, P.gV,
                                                (k == 1 && first_exact) ? 1 : 0, eps, K, 0,
                                                status, lib_capped);
      QTT_LAUNCH_CHECK();
    } else {
      rc = stream_pass(1, cur, M, mcap, ranks, k, n, &np, &ps, ell, seed, P, s);
      if (rc) return rc;
      rc = launch_reduce(P.partials, ps, np, mcap * ell, P.y, s);
      if (rc) return rc;
      k_mqr<<<1, kEigThreads, lds_mqr(), s>>>(P.y, M, ranks, k, ell, P.q1, P.q, P.iq);
      QTT_LAUNCH_CHECK();
      rc = stream_pass(2, cur, M, mcap, ranks, k, n, &np, &ps, ell, seed, P, s);
      if (rc) return rc;
      rc = launch_reduce(P.partials, ps, np, ell * ell, P.gramb, s);
      if (rc) return rc;
      k_meig<<<1, kEigThreads, lds_meig(), s>>>(P.gramb, M, ranks, k, 1, P.q, P.iq, P.scal,
                                                cap[k], cores, off, P.umat, P.gV, 0, eps,
                                                K, 0, status, lib_capped);
      QTT_LAUNCH_CHECK();
    }
    {
      const int rcap = cap[k] < mcap ? cap[k] : mcap;  // bound on r_k
      int tc = mtile(mcap, 64, 512);
      const int as_cap = tc * mcap;
      const size_t lds = sizeof(double) * ((size_t)as_cap + (size_t)mcap * rcap);
      if (lds > (size_t)kMaxStreamLds) return QTT_EINVAL;
      const long long ntile = (n + tc - 1) / tc;
      const int blocks = (int)(ntile < 2048 ? ntile : 2048);
      k_mproj<<<blocks, 256, lds, s>>>(cur, M, ranks, k, n, tc, as_cap, P.umat, P.rbuf[bi]);
      QTT_LAUNCH_CHECK();
    }
    cur = P.rbuf[bi];
    bi ^= 1;
    off += (long long)cap[k - 1] * M * cap[k];
  }
  k_mlast<<<1, 256, 0, s>>>(cur, M, ranks, K, cores + off);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

}  // namespace qtt

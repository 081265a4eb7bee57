// TT-SVD and the max-rank TT-RSVD of Section 5 (modifications (1) and (2))
// on a tensor of K modes of size M, FP64, index i = i_1 + M (i_2 + M (...)).
//
// Step k works on the remainder R_k: the unfolding A_k (m x n column-major,
// m = M r_{k-1}, n = M^(K-k)) is stored contiguously, A_k(a, c) = R_k[a + m c].
//   exact step:       one streaming pass forms G = A A^T (fixed-order sum of
//                     per-block partials); the eigensolver gives U (m x r),
//                     r by Algorithm 1's rule and the cap;
//   randomised step   (min(M cap_{k-1}, n) > R + p, Algorithms 4 and 5):
//                     Y = A Omega (m x ell, Omega drawn on the fly), Q = an
//                     orthonormal basis of range(Y) (eigenvectors of Y^T Y,
//                     one Newton-Schulz polishing step), a second pass forms
//                     G_B = (Q^T A)(Q^T A)^T, its eigenvectors U~ give U = Q U~;
//   both:             R_{k+1} = U^T A (r x n), which is the next unfolding.
// Core k is U read as (r_{k-1}, M, r_k): core[a][i][b] = U[a + r_{k-1} i][b].
#include <math.h>

#include "qtt_eig.hpp"
#include "qtt_internal.hpp"
#include "qtt_philox.hpp"

namespace qtt {

constexpr int kMcTile = 32;      // columns of A per tile of the projection and G_B passes
// columns per tile of the Gram and sketch passes: about 256 / UT, so that a
// tile carries several KB whatever the row count
template <int UT>
constexpr int gram_tile() {
  return UT >= 8 ? 32 : 256 / UT;
}
constexpr int kMsMaxEll = 64;    // sketch width limit (ell = R + p)

// ------------------------------------------------------------- Gram pass
// Partial G = A A^T over the column tiles of this block (grid-stride).
// Thread (ty, tx) owns rows ty + 16u, columns tx + 16v (u, v < UT).
template <int UT>
__global__ void __launch_bounds__(256) k_mgram(const double* R, int M, const int32_t* ranks, int k,
                                               long long n, double* partials, int pstride) {
  constexpr int LDA = 16 * UT + 1;
  constexpr int TC = gram_tile<UT>();
  __shared__ double As[TC * LDA];
  const int m = M * ranks[k - 1];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double acc[UT][UT];
#pragma unroll
  for (int u = 0; u < UT; ++u)
#pragma unroll
    for (int v = 0; v < UT; ++v) acc[u][v] = 0.0;
  // rows m .. 16 UT - 1 of the tile stay zero
  for (int e = tid; e < TC * LDA; e += 256) As[e] = 0.0;
  const long long ntile = (n + TC - 1) / TC;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * TC;
    const int nc = (int)((n - c0) < TC ? (n - c0) : TC);
    __syncthreads();
    for (int e = tid; e < m * TC; e += 256) {
      const int c = e / m, a = e - c * m;
      As[c * LDA + a] = (c < nc) ? R[(long long)m * c0 + e] : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < TC; ++c) {
      double xa[UT], xb[UT];
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        xa[u] = As[c * LDA + ty + 16 * u];
        xb[u] = As[c * LDA + tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < UT; ++u)
#pragma unroll
        for (int v = 0; v < UT; ++v) acc[u][v] = fma(xa[u], xb[v], acc[u][v]);
    }
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int u = 0; u < UT; ++u)
#pragma unroll
    for (int v = 0; v < UT; ++v) {
      const int a = ty + 16 * u, b = tx + 16 * v;
      if (a < m && b < m) P[a * m + b] = acc[u][v];
    }
}

// ----------------------------------------------------------- sketch pass
// Partial Y = A Omega (m x ell, row-major) over this block's column tiles;
// Omega[c][j] = omega_entry(c, j, k, seed) for the global column c.
template <int UT>
__global__ void __launch_bounds__(256) k_msketch(const double* R, int M, const int32_t* ranks, int k,
                                                 long long n, int ell, uint32_t s0, uint32_t s1,
                                                 double* partials, int pstride) {
  constexpr int LDA = 16 * UT + 1;
  constexpr int TC = gram_tile<UT>() < 64 ? gram_tile<UT>() : 64;
  __shared__ double As[TC * LDA];
  __shared__ double Om[TC * kMsMaxEll];
  const int m = M * ranks[k - 1];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  double acc[UT][4];
#pragma unroll
  for (int u = 0; u < UT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int e = tid; e < TC * LDA; e += 256) As[e] = 0.0;
  const long long ntile = (n + TC - 1) / TC;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * TC;
    const int nc = (int)((n - c0) < TC ? (n - c0) : TC);
    __syncthreads();
    for (int e = tid; e < m * TC; e += 256) {
      const int c = e / m, a = e - c * m;
      As[c * LDA + a] = (c < nc) ? R[(long long)m * c0 + e] : 0.0;
    }
    for (int e = tid; e < TC * kMsMaxEll; e += 256) {
      const int c = e / kMsMaxEll, j = e - c * kMsMaxEll;
      Om[e] = (c < nc && j < ell) ? omega_entry(c0 + c, j, k, s0, s1) : 0.0;
    }
    __syncthreads();
    for (int c = 0; c < TC; ++c) {
      double xa[UT], om[4];
#pragma unroll
      for (int u = 0; u < UT; ++u) xa[u] = As[c * LDA + ty + 16 * u];
#pragma unroll
      for (int v = 0; v < 4; ++v) om[v] = Om[c * kMsMaxEll + tx + 16 * v];
#pragma unroll
      for (int u = 0; u < UT; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(xa[u], om[v], acc[u][v]);
    }
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int u = 0; u < UT; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ty + 16 * u, j = tx + 16 * v;
      if (a < m && j < ell) P[a * ell + j] = acc[u][v];
    }
}

// ---------------------------------------------------- G_B = (Q^T A)(Q^T A)^T
// Q: m x q row-major (q = iq[0] <= 64).  Per tile B = Q^T A (q x 32) in LDS,
// then the partial q x q Gram; thread (ty, tx) owns rows ty + 16u, columns
// tx + 16v (u, v < 4).
template <int UT>
__global__ void __launch_bounds__(256) k_mbgram(const double* R, int M, const int32_t* ranks, int k,
                                                long long n, const double* Q, const int32_t* iq,
                                                double* partials, int pstride) {
  constexpr int LDA = 16 * UT + 1;
  constexpr int LB = kMcTile + 1;
  extern __shared__ double sm[];
  double* As = sm;                        // kMcTile x LDA
  double* Qs = As + kMcTile * LDA;        // m x q
  double* Bt = Qs + 16 * UT * kMsMaxEll;  // q x LB
  const int m = M * ranks[k - 1];
  const int q = iq[0];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int e = tid; e < m * q; e += 256) Qs[e] = Q[e];
  // rows q .. 63 of B stay zero
  for (int e = tid; e < kMsMaxEll * LB; e += 256) Bt[e] = 0.0;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  const long long ntile = (n + kMcTile - 1) / kMcTile;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * kMcTile;
    const int nc = (int)((n - c0) < kMcTile ? (n - c0) : kMcTile);
    __syncthreads();
    for (int e = tid; e < m * kMcTile; e += 256) {
      const int c = e / m, a = e - c * m;
      As[c * LDA + a] = (c < nc) ? R[(long long)m * c0 + e] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < q * kMcTile; e += 256) {
      const int j = e / kMcTile, c = e - j * kMcTile;
      double s0 = 0.0, s1 = 0.0;
      int a = 0;
      for (; a + 1 < m; a += 2) {
        s0 = fma(Qs[a * q + j], As[c * LDA + a], s0);
        s1 = fma(Qs[(a + 1) * q + j], As[c * LDA + a + 1], s1);
      }
      if (a < m) s0 = fma(Qs[a * q + j], As[c * LDA + a], s0);
      Bt[j * LB + c] = s0 + s1;
    }
    __syncthreads();
    for (int c = 0; c < kMcTile; ++c) {
      double xa[4], xb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xa[u] = Bt[(ty + 16 * u) * LB + c];
        xb[u] = Bt[(tx + 16 * u) * LB + c];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(xa[u], xb[v], acc[u][v]);
    }
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = ty + 16 * u, b = tx + 16 * v;
      if (a < q && b < q) P[a * q + b] = acc[u][v];
    }
}

// -------------------------------------------------------- eigen problems
struct MEig {
  double *A, *V, *lam, *sx;
  int *perm, *iscr;
  int lda;
};

__device__ __forceinline__ MEig meig_layout(double* smem, int E, double* gA, double* gV) {
  MEig L;
  if (E <= kEigLds) {
    L.lda = kEigLds + 1;
    L.A = smem;
    L.V = L.A + L.lda * L.lda;
    L.lam = L.V + L.lda * L.lda;
  } else {
    L.lda = kMaxM + 1;
    L.A = gA;
    L.V = gV;
    L.lam = smem;
  }
  L.sx = L.lam + kMaxM + 8;
  L.perm = (int*)(L.sx + kEigScratch);
  L.iscr = L.perm + kMaxM + 8;
  return L;
}

template <class MP>
__device__ int meig_solve(const MEig& L, MP A, MP V, int E, double tau2, int cap, int32_t* rk,
                          int k) {
  StepOut so;
  so.ranks = rk;
  so.status = nullptr;
  so.sv = nullptr;
  so.lib_capped = 0;
  so.dbg = nullptr;
  so.delta2 = 0.0;
  return solve_and_truncate<kEigThreads, true>(A, V, E, L.lda, lds(L.sx), lds(L.iscr), lds(L.lam),
                                              lds(L.perm), tau2, cap, k, so);
}

// Step k's truncated eigendecomposition.  Exact step (use_q = 0): G is m x m
// and U = V[:, :r].  Randomised step (use_q = 1): G is G_B (q x q) and
// U = Q V[:, :r].  Writes ranks[k], core k and U (m x r, row-major) to umat.
__global__ void __launch_bounds__(kEigThreads) k_meig(const double* G, int M, int32_t* ranks,
                                                      int k, int use_q, const double* Q,
                                                      const int32_t* iq, double* scal,
                                                      int cap_k, double* cores, long long off_k,
                                                      double* umat, double* gA, double* gV,
                                                      int set_tau, double eps, int K) {
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int rp = ranks[k - 1];
  const int m = M * rp;
  const int q = use_q ? iq[0] : m;
  const int E = q;
  const MEig L = meig_layout(smem, E, gA, gV);
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
  __syncthreads();
  int r;
  if (E <= kEigLds)
    r = meig_solve(L, lds(L.A), lds(L.V), E, scal[1], cap_k, ranks, k);
  else
    r = meig_solve(L, L.A, L.V, E, scal[1], cap_k, ranks, k);
  // U (m x r) and core k
  for (int e = tid; e < m * r; e += kEigThreads) {
    const int b = e % r, t = e / r;
    const int i = t % M, ai = t / M;   // core order (r_{k-1}, M, r_k)
    const int row = ai + rp * i;       // unfolding row of that entry
    const int col = L.perm[b];
    double u;
    if (use_q) {
      u = 0.0;
      for (int c = 0; c < q; ++c) u = fma(Q[row * q + c], L.V[c * L.lda + col], u);
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
__global__ void __launch_bounds__(kEigThreads) k_mqr(const double* Y, int M, const int32_t* ranks,
                                                     int k, int ell, double* Q1, double* Q,
                                                     int32_t* iq) {
  extern __shared__ double smem[];
  __shared__ int32_t rk[4];
  __shared__ double Sq[kMsMaxEll * kMsMaxEll];
  const int tid = threadIdx.x;
  const int m = M * ranks[k - 1];
  const int E = ell;  // <= 64: LDS
  const MEig L = meig_layout(smem, E, nullptr, nullptr);
  for (int e = tid; e < E * E; e += kEigThreads) {
    const int a = e / E, b = e - a * E;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(Y[i * ell + a], Y[i * ell + b], s);
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
      for (int c = 0; c < ell; ++c) s = fma(Y[i * ell + c], L.V[c * L.lda + L.perm[b]], s);
      Q1[e] = s / sqrt(L.lam[b]);
    }
  }
  __syncthreads();
  // S = (3I - Q1^T Q1) / 2
  for (int e = tid; e < qn * qn; e += kEigThreads) {
    const int a = e / qn, b = e - a * qn;
    double s = 0.0;
    for (int i = 0; i < m; ++i) s = fma(Q1[i * qn + a], Q1[i * qn + b], s);
    Sq[e] = (a == b ? 1.5 : 0.0) - 0.5 * s;
  }
  __syncthreads();
  for (int e = tid; e < m * qn; e += kEigThreads) {
    const int i = e / qn, b = e - i * qn;
    double s = 0.0;
    for (int c = 0; c < qn; ++c) s = fma(Q1[i * qn + c], Sq[c * qn + b], s);
    Q[e] = s;
  }
  if (tid == 0) iq[0] = qn;
}

// ------------------------------------------------------------ projection
// R_{k+1}[b + r c] = sum_a U[a][b] A(a, c); U (m x r, row-major) in LDS.
__global__ void __launch_bounds__(256) k_mproj(const double* R, int M, const int32_t* ranks, int k,
                                               long long n, const double* U, double* Rn, int TC) {
  extern __shared__ double sm[];
  const int m = M * ranks[k - 1];
  const int r = ranks[k];
  const int LDA = m + 1;
  double* Us = sm;                   // m x r
  double* As = Us + kMaxM * kMaxRank;  // TC x LDA
  const int tid = threadIdx.x;
  for (int e = tid; e < m * r; e += 256) Us[e] = U[e];
  const long long ntile = (n + TC - 1) / TC;
  for (long long t = blockIdx.x; t < ntile; t += gridDim.x) {
    const long long c0 = t * TC;
    const int nc = (int)((n - c0) < TC ? (n - c0) : TC);
    __syncthreads();
    for (int e = tid; e < m * nc; e += 256) {
      const int c = e / m, a = e - c * m;
      As[c * LDA + a] = R[(long long)m * c0 + e];
    }
    __syncthreads();
    for (int e = tid; e < r * nc; e += 256) {
      const int c = e / r, b = e - c * r;
      double s0 = 0.0, s1 = 0.0;
      int a = 0;
      for (; a + 1 < m; a += 2) {
        s0 = fma(Us[a * r + b], As[c * LDA + a], s0);
        s1 = fma(Us[(a + 1) * r + b], As[c * LDA + a + 1], s1);
      }
      if (a < m) s0 = fma(Us[a * r + b], As[c * LDA + a], s0);
      Rn[(long long)r * c0 + e] = s0 + s1;
    }
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
  double *scal, *dotp, *partials, *gram, *gramb, *y, *umat, *q1, *q, *gA, *gV, *rbuf[2];
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
  p.partials = ar.take<double>((size_t)kMaxPartials * p.pstride);
  p.gram = ar.take<double>((size_t)kMaxM * kMaxM);
  p.gramb = ar.take<double>((size_t)kMsMaxEll * kMsMaxEll);
  p.y = ar.take<double>((size_t)kMaxM * kMsMaxEll);
  p.umat = ar.take<double>((size_t)kMaxM * kMaxRank);
  p.q1 = ar.take<double>((size_t)kMaxM * kMsMaxEll);
  p.q = ar.take<double>((size_t)kMaxM * kMsMaxEll);
  p.gA = ar.take<double>((size_t)(kMaxM + 1) * (kMaxM + 1));
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

static size_t lds_meig() {
  const int lda = kEigLds + 1;
  return sizeof(double) * (2 * lda * lda + (kMaxM + 8) + kEigScratch) +
         sizeof(int) * (kMaxM + 8 + 8 + 256);
}

// projection tile: more columns when the unfolding has few rows
static int proj_tile(int mcap) { return mcap <= 16 ? 256 : (mcap <= 32 ? 128 : (mcap <= 64 ? 64 : 32)); }

static size_t lds_mproj() {
  return sizeof(double) * ((size_t)kMaxM * kMaxRank + (size_t)256 * 17);
}

template <int UT>
static size_t lds_mbgram() {
  return sizeof(double) * ((size_t)kMcTile * (16 * UT + 1) + (size_t)16 * UT * kMsMaxEll +
                           (size_t)kMsMaxEll * (kMcTile + 1));
}

template <int UT>
static void set_mbgram_attr() {
  (void)hipFuncSetAttribute((const void*)k_mbgram<UT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)lds_mbgram<UT>());
}

template <int UT>
static void launch_stream_passes(int which, const double* R, int M, int32_t* ranks, int k,
                                 long long n, int blocks, int ell, uint64_t seed,
                                 const ModesPlan& P, hipStream_t s) {
  if (which == 0) {
    k_mgram<UT><<<blocks, 256, 0, s>>>(R, M, ranks, k, n, P.partials, P.pstride);
  } else if (which == 1) {
    k_msketch<UT><<<blocks, 256, 0, s>>>(R, M, ranks, k, n, ell, (uint32_t)(seed & 0xFFFFFFFFu),
                                         (uint32_t)(seed >> 32), P.partials, P.pstride);
  } else {
    k_mbgram<UT><<<blocks, 256, lds_mbgram<UT>(), s>>>(R, M, ranks, k, n, P.q, P.iq, P.partials, P.pstride);
  }
}

static int stream_pass(int which, const double* R, int M, int mcap, int32_t* ranks, int k,
                       long long n, int* nparts, int* pstride, int ell, uint64_t seed,
                       const ModesPlan& P, hipStream_t s) {
  // partials of sz doubles each, as many as the partials buffer holds (<= 1024)
  const long long sz = which == 0 ? (long long)mcap * mcap
                                  : (which == 1 ? (long long)mcap * ell : (long long)ell * ell);
  const long long cap_parts = (long long)kMaxPartials * P.pstride / sz;
  const long long ntile = (n + kMcTile - 1) / kMcTile;
  long long b = ntile < 1024 ? ntile : 1024;
  if (b > cap_parts) b = cap_parts;
  const int blocks = (int)(b < 1 ? 1 : b);
  *nparts = blocks;
  *pstride = (int)sz;
  ModesPlan Q = P;
  Q.pstride = (int)sz;
  const int ut = (mcap + 15) / 16;
  switch (ut) {
    case 1: launch_stream_passes<1>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    case 2: launch_stream_passes<2>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    case 3: launch_stream_passes<3>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    case 4: launch_stream_passes<4>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    case 5: launch_stream_passes<5>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    case 6: launch_stream_passes<6>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    case 7: launch_stream_passes<7>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
    default: launch_stream_passes<8>(which, R, M, ranks, k, n, blocks, ell, seed, Q, s); break;
  }
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_decompose_modes(const double* x, int K, int M, double eps, int method, int oversample,
                        uint64_t seed, const int32_t* cap, int32_t* ranks, double* cores,
                        void* ws, hipStream_t s) {
  static bool attrs = false;
  if (!attrs) {
    (void)hipFuncSetAttribute((const void*)k_meig, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds_meig());
    (void)hipFuncSetAttribute((const void*)k_mqr, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds_meig());
    (void)hipFuncSetAttribute((const void*)k_mproj, hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)lds_mproj());
    set_mbgram_attr<1>();
    set_mbgram_attr<2>();
    set_mbgram_attr<3>();
    set_mbgram_attr<4>();
    set_mbgram_attr<5>();
    set_mbgram_attr<6>();
    set_mbgram_attr<7>();
    set_mbgram_attr<8>();
    attrs = true;
  }
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
    if (!rs) {
      rc = stream_pass(0, cur, M, mcap, ranks, k, n, &np, &ps, 0, seed, P, s);
      if (rc) return rc;
      rc = launch_reduce(P.partials, ps, np, mcap * mcap, P.gram, s);
      if (rc) return rc;
      k_meig<<<1, kEigThreads, lds_meig(), s>>>(P.gram, M, ranks, k, 0, nullptr, P.iq, P.scal,
                                                cap[k], cores, off, P.umat, P.gA, P.gV,
                                                (k == 1 && first_exact) ? 1 : 0, eps, K);
      QTT_LAUNCH_CHECK();
    } else {
      rc = stream_pass(1, cur, M, mcap, ranks, k, n, &np, &ps, ell, seed, P, s);
      if (rc) return rc;
      rc = launch_reduce(P.partials, ps, np, mcap * ell, P.y, s);
      if (rc) return rc;
      k_mqr<<<1, kEigThreads, lds_meig(), s>>>(P.y, M, ranks, k, ell, P.q1, P.q, P.iq);
      QTT_LAUNCH_CHECK();
      rc = stream_pass(2, cur, M, mcap, ranks, k, n, &np, &ps, ell, seed, P, s);
      if (rc) return rc;
      rc = launch_reduce(P.partials, ps, np, ell * ell, P.gramb, s);
      if (rc) return rc;
      k_meig<<<1, kEigThreads, lds_meig(), s>>>(P.gramb, M, ranks, k, 1, P.q, P.iq, P.scal,
                                                cap[k], cores, off, P.umat, P.gA, P.gV, 0, eps,
                                                K);
      QTT_LAUNCH_CHECK();
    }
    {
      const int tc = proj_tile(mcap);
      const long long ntile = (n + tc - 1) / tc;
      const int blocks = (int)(ntile < 2048 ? ntile : 2048);
      k_mproj<<<blocks, 256, lds_mproj(), s>>>(cur, M, ranks, k, n, P.umat, P.rbuf[bi], tc);
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

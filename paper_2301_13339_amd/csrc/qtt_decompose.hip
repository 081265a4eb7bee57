// TT-SVD sweep (Algorithm 1 with the max-rank modification (1)) on gfx950.
//
// Notation.  For step k (1..D-1) the remainder X_k is an n_k x m_k row-major
// matrix, n_k = 2^(D-k), m_k = 2 r_{k-1}; its column c = a + r_{k-1} i_k is
// the row of the paper's unfolding A^{k} (Lemma 5.1), so X_k = (A^{k})^T and
// the left singular vectors of A^{k} are the eigenvectors of X_k^T X_k.  With
// U_k the kept eigenvectors, core k is U_k reshaped (r_{k-1}, 2, r_k) and the
// next remainder X_{k+1} is the memory of X_k U_k (n_k x r_k) read as an
// (n_k/2) x (2 r_k) matrix -- the reshape is free in row-major order.
//
// Schedule (D modes, N = 2^D samples):
//  * N <= kTailElems: one workgroup holds the samples in LDS and runs the
//    whole sweep (k_tail).
//  * otherwise
//    - k_level_gram streams the samples once and forms the 64 x 64 Gram of
//      the data viewed as (N/64) x 64 (FP64, per-block partials);
//    - k_level_eig runs steps 1..6 from it: the Gram of X_k is
//      P_k^T G_k P_k, G_k a block sum of the 64 x 64 Gram and P_k the
//      block-diagonal embedding of the left interface Phi_{k-1};
//    - k_project_gram computes X_{k+1} = X_k U_k block by block and the
//      partial Grams of X_{k+1} in the same pass (one read, one write);
//    - k_reduce sums the partials in a fixed order (deterministic);
//    - k_eig_step solves one step;
//    - once X_k fits kTailElems, k_tail finishes in LDS (dual Gram X X^T
//      when n_k < m_k).
// Ranks stay in device memory; no kernel needs a host synchronisation.
#include <math.h>

#include <mutex>

#include "qtt_eig.hpp"
#include "qtt_internal.hpp"
#include "qtt_sinc.hpp"

namespace qtt {

// ------------------------------------------------------------ sample access
// GEN = 0: stored samples x[u].
// GEN = 1: generator of the sinc-kernel Toeplitz vector, unnormalised (the
//          last core is divided by the sample sum afterwards).
// GEN = 2: derivative of the normalised generator with respect to the
//          bandwidth, (s'_m - s_m S'/S) / S, with c = (1/S, S'/S) read from
//          the device array passed in place of the samples.
template <typename T, int GEN>
__device__ __forceinline__ double sample(const T* x, long long u, double B, int nk) {
  if (GEN == 1) return sinc_gen(u, B, nk);
  if (GEN == 2) {
    const double* c = reinterpret_cast<const double*>(x);
    double sv, dv;
    sinc_gen_pair(u, B, nk, &sv, &dv);
    return (dv - sv * c[1]) * c[0];
  }
  return (double)x[u];
}

__device__ __forceinline__ int finite_d(double v) { return isfinite(v) ? 1 : 0; }

// write core k (1-based) from U (m x r, row-major, rows c = a + rp*i)
template <typename T>
__device__ void write_core_from_u(T* cores, long long off, const double* U, int ldu, int rp, int r,
                                  int tid, int nt) {
  const int total = rp * 2 * r;
  for (int e = tid; e < total; e += nt) {
    const int b = e % r;
    const int ai = e / r;
    const int i = ai & 1, a = ai >> 1;
    cores[off + e] = (T)U[(a + rp * i) * ldu + b];
  }
}

// ----------------------------------------------------------------- D == 1
template <typename T, int GEN>
__global__ void k_single(const T* x, double B, int nk, T* cores, int32_t* ranks, double* scal,
                         int32_t* status) {
  if (threadIdx.x == 0) {
    const double v0 = sample<T, GEN>(x, 0, B, nk), v1 = sample<T, GEN>(x, 1, B, nk);
    double s = (GEN == 1) ? v0 + v1 : 1.0;
    if (s == 0.0) s = 1.0;
    cores[0] = (T)(v0 / s);
    cores[1] = (T)(v1 / s);
    ranks[0] = 1;
    ranks[1] = 1;
    if (status && !(finite_d(v0) && finite_d(v1))) atomicOr(status, QTT_STATUS_NONFINITE);
    scal[0] = v0 * v0 + v1 * v1;
  }
}

// ------------------------------------------------------------ level Gram
// Gram of the samples viewed as rows x 64 (row-major), 256 threads: thread
// (ty, tx) accumulates the 4 x 4 tile rows 4ty.., cols 4tx.. over the 32-row
// stages bid, bid + nblk, ... (st: 32 x 64 doubles of LDS).  Also the sum of
// the samples (generator normalisation) and a finiteness flag.
template <typename T, int GEN>
__device__ __forceinline__ void level_gram_acc(const T* x, double B, int nk, long long rows,
                                               long long bid, long long nblk, double* st,
                                               double (&acc)[4][4], double& gsum, int& fin) {
  constexpr int W = 64, SR = 32;
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  gsum = 0.0;
  fin = 1;
  const long long nstage = (rows + SR - 1) / SR;
  // the next stage is read into registers while the current one is summed
  constexpr int PER = SR * W / 256;
  double pre[PER];
  auto fetch = [&](long long sidx) {
    const long long r0 = sidx * SR;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = tid + 256 * j;
      pre[j] = (r0 + e / W < rows) ? sample<T, GEN>(x, r0 * W + e, B, nk) : 0.0;
    }
  };
  if (bid < nstage) fetch(bid);
  for (long long sidx = bid; sidx < nstage; sidx += nblk) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const double v = pre[j];
      fin &= finite_d(v);
      gsum += v;
      st[tid + 256 * j] = v;
    }
    __syncthreads();
    if (sidx + nblk < nstage) fetch(sidx + nblk);
    for (int rr = 0; rr < SR; ++rr) {
      double xa[4], xb[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xa[a] = st[rr * W + 4 * ty + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) xb[b] = st[rr * W + 4 * tx + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(xa[a], xb[b], acc[a][b]);
    }
    __syncthreads();
  }
}

// fixed-order workgroup sum (red: 256 doubles of LDS); every thread gets it
__device__ __forceinline__ double wg_sum256(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double t = red[0];
  __syncthreads();
  return t;
}

// Partial Grams over the stages of this block (one partial per block).
template <typename T, int GEN>
__global__ void __launch_bounds__(256) k_level_gram(const T* x, double B, int nk, long long rows,
                                                    double* partials, int pstride,
                                                    double* gsum_part, int32_t* iflags) {
  constexpr int W = 64, SR = 32;
  __shared__ double st[SR * W];
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  double acc[4][4];
  double gsum;
  int fin;
  level_gram_acc<T, GEN>(x, B, nk, rows, blockIdx.x, gridDim.x, st, acc, gsum, fin);
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) P[(4 * ty + a) * W + 4 * tx + b] = acc[a][b];
  const double tot = wg_sum256(gsum, red);
  if (tid == 0) gsum_part[blockIdx.x] = tot;
  if (!fin) atomicOr(iflags, 1);
}

// --------------------------------------------------------------- reduction
// out[e] = sum_b partials[b*pstride + e] for e < count.  Block of 256 threads
// = 64 entries x 4 partial groups; group g sums partials g, g+4, ... and the
// four group sums are added in a fixed order (deterministic).  Block 0 also
// sums the generator partial sums into scal[2].  With mranks, the entries
// are an M x M Gram at row stride mstride, M = 2 mranks[mk - 1] on the
// device, and entries outside it (never written by the pass) are skipped.
__global__ void __launch_bounds__(256) k_reduce(const double* partials, int pstride, int nparts,
                                                int count, double* out, const double* gsum_part,
                                                double* scal, const int32_t* mranks = nullptr,
                                                int mk = 0, int mstride = 1) {
  __shared__ double red[4][64];
  const int el = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  double s = 0.0;
  bool in = e < count;
  if (mranks) {
    const int M = 2 * mranks[mk - 1];
    const int row = e / mstride, col = e - row * mstride;
    in = in && row < M && col < M;
  }
  if (in) {
    // eight independent loads in flight per thread, summed in a fixed order
    int b = g;
    for (; b + 28 < nparts; b += 32) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partials[(size_t)(b + 4 * u) * pstride + e];
      s += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    for (; b < nparts; b += 4) s += partials[(size_t)b * pstride + e];
  }
  red[g][el] = s;
  __syncthreads();
  if (g == 0 && in) out[e] = (red[0][el] + red[1][el]) + (red[2][el] + red[3][el]);
  if (gsum_part && blockIdx.x == 0 && threadIdx.x < 64) {  // uniform in the wave
    // the squared norm: every lane sums a stride of the block partials, then
    // a butterfly over the wave; each lane's order is fixed, lane 0's is kept
    double t = 0.0;
    for (int b = threadIdx.x; b < nparts; b += 64) t += gsum_part[b];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
    if (threadIdx.x == 0) scal[2] = t;
  }
}

// k_reduce for other translation units (out[e] = sum_b partials[b * pstride + e])
int launch_reduce(const double* partials, int pstride, int nparts, int count, double* out,
                  hipStream_t s) {
  k_reduce<<<(count + 63) / 64, 256, 0, s>>>(partials, pstride, nparts, count, out, nullptr,
                                             nullptr);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

// ------------------------------------------------------ small LDS products
// C (M x N) = A (M x K) B (K x N) with all operands in LDS: A(i, k) =
// A[i*ai + k*ak], B(k, j) = B[k*bk + j*bj]; store(i, j, v) receives the
// results.  On the FP64 matrix cores: 16 x 16 blocks of C spread
// over the four waves, and for each block the operands of sixteen k loaded
// before four MFMAs (v_mfma_f64_16x16x4f64: lane (lk, lr) supplies
// A(16 bi + lr, k + lk) and B(k + lk, 16 bj + lr) and receives
// C(16 bi + 4 e + lk, 16 bj + lr) in element e).  Operands outside M, N, K
// enter as zeros.
template <class F>
__device__ __forceinline__ void lds_gemm_mfma(int M, int N, int K, lds_ptr<const double> A,
                                              int ai, int ak, lds_ptr<const double> B, int bk,
                                              int bj, F store) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
  const int mb = (M + 15) >> 4, nb = (N + 15) >> 4;
  for (int blk = w; blk < mb * nb; blk += 4) {  // wave-uniform
    const int bi = blk / nb, bjb = blk - bi * nb;
    const int row = 16 * bi + lr, col = 16 * bjb + lr;
    const bool rin = row < M, cin = col < N;
    const int rc = rin ? row : 0, cc = cin ? col : 0;
    syev_f64x4 acc = syev_f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k16 = 0; k16 < K; k16 += 16) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k16 + 4 * u + lk;
        const bool kin = kk < K;
        const int kc = kin ? kk : 0;
        const double a = A[rc * ai + kc * ak];
        const double b = B[kc * bk + cc * bj];
        av[u] = (rin & kin) ? a : 0.0;
        bv[u] = (cin & kin) ? b : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * bi + 4 * e + lk, j = 16 * bjb + lr;
      if (i < M && j < N) store(i, j, acc[e]);
    }
  }
}

// ------------------------------------------------------------- level eig
// Steps 1..L from the Gram GZ (64 x 64, at the start of smem) of the samples
// viewed as (N/64) x 64.  Writes cores 1..L, ranks 0..L, tau^2 (scal[1]) and
// Phi_L (64 x r_L) to umat.
template <typename T>
__device__ void level_steps(double* smem, int L, int D, double eps, const Meta& meta, T* cores,
                            double* scal, double* umat, const StepOut& so) {
  constexpr int NT = kEigThreads, W = 64, LDA = 65;
  double* GZ = smem;                 // 64*64
  double* A = GZ + W * W;            // 65*65
  double* V = A + LDA * LDA;         // 65*65
  double* T1 = V + LDA * LDA;        // 64*64 (also Phi_k scratch)
  double* Phi = T1 + W * W;          // 32*32
  double* lam = Phi + 32 * 32;       // 72
  double* sx = lam + 72;             // kEigScratch
  int* perm = (int*)(sx + kEigScratch);  // 72
  int* iscr = perm + 72;
  const int tid = threadIdx.x;
  if (tid == 0) {
    Phi[0] = 1.0;
    so.ranks[0] = 1;
  }
  __syncthreads();
  double nrm2 = 0.0;
  for (int i = 0; i < W; ++i) nrm2 += GZ[i * W + i];
  const double tau2 = (D > 1) ? eps * eps * nrm2 / (double)(D - 1) : 0.0;
  if (tid == 0) {
    scal[0] = nrm2;
    scal[1] = tau2;
  }
  // Full-rank pre-test of steps 1 .. min(L, 5).  While every earlier step
  // keeps its full rank 2^(k-1) with U = I, Phi_{k-1} and P_k are
  // permutations, so the matrix A of step k is G_k with rows and columns
  // permuted: A - mu I is positive definite exactly when G_k - mu I is, and
  // the trace that mu takes is the same.  The tests of these steps are then
  // independent and run on separate waves (step 5 on wave 0, 4 on wave 1, 3
  // on wave 2, 2 and 1 on wave 3).  The leading steps that pass keep V = I
  // without forming A or solving; the first that fails, and every later
  // one, take the usual path.  Not with singular values or a drop-off
  // requested (those need the eigenvalues).
  int npre = 0;
  const int KP = L < 5 ? L : 5;
  if (!so.sv && !(so.delta2 > 0.0)) {
    double* Gs = A;                      // slots of 32 x 32 (lda 32) over A and V
    ldsi okf = lds(perm);                // okf[k]: step k passed (perm is free here)
    for (int k = 1; k <= KP; ++k) {
      const int w = 1 << k, reps = W / w;
      for (int e = tid; e < w * w; e += NT) {
        const int c = e / w, c2 = e - c * w;
        double g = 0.0;
        for (int h = 0; h < reps; ++h) g += GZ[(c + h * w) * W + c2 + h * w];
        Gs[(k - 1) * 1024 + c * 32 + c2] = g;
      }
    }
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(tid >> 6), l = tid & 63;
    ldsd cb = lds(A + 5 * 1024 + 64 * q);  // per-wave Cholesky buffer
    auto test = [&](int k) {
      const int E = 1 << k;
      const lds_ptr<const double> G = lds<const double>(Gs + (k - 1) * 1024);
      double tr = 0.0;
      for (int i = l; i < E; i += 64) tr += G[i * 32 + i];
      tr = sum64(tr);
      const bool ok = isfinite(tr) && meta.caps[k] >= E &&
                      chol_pd_wave(G, E, 32, tau2 * (1.0 + 1e-6) + 1e-12 * tr, cb);
      if (l == 0) okf[k] = ok ? 1 : 0;
    };
    if (q == 0) {
      if (KP >= 5) test(5);
    } else if (q == 1) {
      if (KP >= 4) test(4);
    } else if (q == 2) {
      if (KP >= 3) test(3);
    } else {
      if (KP >= 2) test(2);
      test(1);
    }
    __syncthreads();
    while (npre < KP && okf[npre + 1]) ++npre;
    __syncthreads();  // perm is rewritten by the steps
  }
  int rp = 1;  // r_{k-1}
  for (int k = 1; k <= L; ++k) {
#ifdef QTT_EIG_TIMING
    const long long ls0 = wall_clock64();
#endif
    const int w = 1 << k, half = w >> 1;
    const int m = 2 * rp;
    int r;
#ifdef QTT_EIG_TIMING
    long long ls1, ls2;
#endif
    if (k <= npre) {  // rank m by the pre-test: V = I in the identity order
      for (int i = tid; i < m; i += NT) perm[i] = i;
      for (int idx = tid; idx < m * m; idx += NT) {
        const int a = idx / m, c = idx - a * m;
        V[a * LDA + c] = (a == c) ? 1.0 : 0.0;
      }
      if (tid == 0) so.ranks[k] = m;
      __syncthreads();
      r = m;
#ifdef QTT_EIG_TIMING
      ls1 = ls2 = wall_clock64();
#endif
    } else {
      // G_k[c][c'] = sum_h GZ[c + h w][c' + h w]  (w x w, into V before the solve)
      const int reps = W / w;
      for (int e = tid; e < w * w; e += NT) {
        const int c = e / w, c2 = e - c * w;
        double g = 0.0;
        for (int h = 0; h < reps; ++h) g += GZ[(c + h * w) * W + c2 + h * w];
        V[c * LDA + c2] = g;
      }
      __syncthreads();
      // T1 = G_k P_k (w x m): P_k[cl + half i][i' rp + a] = [i == i'] Phi[cl][a],
      // so column block i of T1 is G_k[:, half i .. half i + half) Phi
      {
        ldsd T1l = lds(T1);
        for (int i = 0; i < 2; ++i)
          lds_gemm_mfma(w, rp, half, lds<const double>(V + half * i), LDA, 1, lds<const double>(Phi), 32, 1,
                   [&](int c, int a, double v) { T1l[c * m + i * rp + a] = v; });
      }
      __syncthreads();
      // A = P_k^T T1 (m x m): row block i is Phi^T T1[half i .. half i + half, :]
      {
        ldsd Al = lds(A);
        for (int i = 0; i < 2; ++i)
          lds_gemm_mfma(rp, m, half, lds<const double>(Phi), 1, 32, lds<const double>(T1 + half * i * m), m,
                   1, [&](int a, int col, double v) { Al[(i * rp + a) * LDA + col] = v; });
      }
      __syncthreads();
#ifdef QTT_EIG_TIMING
      ls1 = wall_clock64();
#endif
      r = solve_and_truncate<NT>(lds(A), lds(V), m, LDA, lds(sx), lds(iscr), lds(lam), lds(perm),
                                 tau2, meta.caps[k], k, so, true, rp == (1 << (k - 1)));
#ifdef QTT_EIG_TIMING
      ls2 = wall_clock64();
#endif
    }
    // core k = V[:, perm[:r]]
    {
      const int total = rp * 2 * r;
      for (int e = tid; e < total; e += NT) {
        const int b = e % r, ai = e / r;
        const int i = ai & 1, a = ai >> 1;
        cores[meta.offs[k - 1] + e] = (T)V[(a + rp * i) * LDA + perm[b]];
      }
    }
    // Phi_k = P_k U_k (w x r) into T1: row block i is Phi U[rp i .. rp i + rp, :]
    // (perm is the identity)
    {
      ldsd T1l = lds(T1);
      for (int i = 0; i < 2; ++i)
        lds_gemm_mfma(half, r, rp, lds<const double>(Phi), 32, 1, lds<const double>(V + rp * i * LDA), LDA,
                 1, [&](int cl, int b, double v) { T1l[(cl + half * i) * r + b] = v; });
    }
    __syncthreads();
    if (k < L) {
      for (int e = tid; e < w * r; e += NT) {
        const int c = e / r, b = e - c * r;
        Phi[c * 32 + b] = T1[e];
      }
    } else {
      for (int e = tid; e < w * r; e += NT) umat[e] = T1[e];
    }
    __syncthreads();
#ifdef QTT_EIG_TIMING
    if (tid == 0 && so.dbg) {
      const long long ls3 = wall_clock64();
      so.dbg[400 + 3 * k] = (int)(ls1 - ls0);
      so.dbg[401 + 3 * k] = (int)(ls2 - ls1);
      so.dbg[402 + 3 * k] = (int)(ls3 - ls2);
    }
#endif
    rp = r;
  }
}

template <typename T>
__global__ void __launch_bounds__(kEigThreads) k_level_eig(const double* gram, int L, int D,
                                                           double eps, const Meta meta,
                                                           T* cores, double* scal, double* umat,
                                                           StepOut so) {
  extern __shared__ double smem[];
  for (int e = threadIdx.x; e < 64 * 64; e += kEigThreads) smem[e] = gram[e];
  __syncthreads();
  level_steps<T>(smem, L, D, eps, meta, cores, scal, umat, so);
}


// --------------------------------------------------------- project + Gram
// Y = A U for A (rowsA x WA, row-major) and U (WA x r); Y is written to Xout
// (row-major, r columns) and is the next remainder, whose rows pair two Y
// rows.  With do_gram, thread (ty, tx) accumulates the TS x TS tile of the
// Gram of the next remainder (2r x 2r) over the 32-row stages bid, bid +
// nblk, ...  smem: WA*r + 32*WA + 32*r doubles.
template <typename T, int GEN, int TS>
__device__ __forceinline__ void project_gram_acc(const T* Ain, double B, int nk, long long rowsA,
                                                 int WA, int r, const double* U, T* Xout,
                                                 int do_gram, long long bid, long long nblk,
                                                 double* smem, double (&acc)[TS][TS]) {
  constexpr int SR = 32;
  const int tid = threadIdx.x;
  const int M = 2 * r;
  double* Us = smem;              // WA*r
  double* As = Us + WA * r;       // SR*WA
  double* Ys = As + SR * WA;      // SR*r
  for (int e = tid; e < WA * r; e += 256) Us[e] = U[e];
  const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int a = 0; a < TS; ++a)
#pragma unroll
    for (int b = 0; b < TS; ++b) acc[a][b] = 0.0;
  __syncthreads();
  const long long nstage = (rowsA + SR - 1) / SR;
  for (long long sidx = bid; sidx < nstage; sidx += nblk) {
    const long long r0 = sidx * SR;
    const int nr = (int)((rowsA - r0) < SR ? (rowsA - r0) : SR);
    for (int e = tid; e < nr * WA; e += 256) As[e] = sample<T, GEN>(Ain, r0 * WA + e, B, nk);
    __syncthreads();
    for (int e = tid; e < nr * r; e += 256) {
      const int row = e / r, col = e - row * r;
      double s = 0.0;
      for (int c = 0; c < WA; ++c) s = fma(As[row * WA + c], Us[c * r + col], s);
      Ys[e] = s;
      Xout[r0 * r + e] = (T)s;
    }
    __syncthreads();
    if (do_gram) {
      const int nx = nr >> 1;
      for (int b = 0; b < nx; ++b) {
        const double* xr = Ys + 2 * b * r;
        double xa[TS], xb[TS];
#pragma unroll
        for (int a = 0; a < TS; ++a) {
          const int i = ty * TS + a;
          xa[a] = i < M ? xr[i] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < TS; ++c) {
          const int j = tx * TS + c;
          xb[c] = j < M ? xr[j] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < TS; ++a)
#pragma unroll
          for (int c = 0; c < TS; ++c) acc[a][c] = fma(xa[a], xb[c], acc[a][c]);
      }
    }
    __syncthreads();
  }
}

// WA is either fixed (wa_fixed > 0) or 2*ranks[kin-1]; one partial Gram
// (square stride mstride) per block.
template <typename T, int GEN, int TS>
__global__ void __launch_bounds__(256) k_project_gram(const T* Ain, double B, int nk,
                                                      long long rowsA, int wa_fixed,
                                                      const int32_t* ranks, int kin,
                                                      const double* U, T* Xout, int do_gram,
                                                      double* partials, int pstride,
                                                      int mstride) {
  extern __shared__ double smem[];
  const int WA = wa_fixed > 0 ? wa_fixed : 2 * ranks[kin - 1];
  const int r = ranks[kin];
  double acc[TS][TS];
  project_gram_acc<T, GEN, TS>(Ain, B, nk, rowsA, WA, r, U, Xout, do_gram, blockIdx.x, gridDim.x,
                               smem, acc);
  if (do_gram) {
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
    double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
    for (int a = 0; a < TS; ++a)
#pragma unroll
      for (int c = 0; c < TS; ++c) {
        const int i = ty * TS + a, j = tx * TS + c;
        if (i < mstride && j < mstride) P[i * mstride + j] = acc[a][c];
      }
  }
}

// The same projection and partial Gram on the FP64 matrix cores.  A stage
// of 32 rows: A (32 x WA) is staged in LDS k-major, Y = A U is formed by
// 16 x 16 blocks (wave w: row block w & 1, column blocks w >> 1, (w >> 1) + 2,
// ...), written to Xout and kept in LDS, and the Gram of the next remainder
// (Y read as 16 x 2r) accumulates in registers, 16 x 16 blocks of the
// 2r x 2r result spread round-robin over the waves.  RB: bound on r (16, 32
// or 64).  v_mfma_f64_16x16x4f64: A entry (row l % 16, k l / 16), B entry
// (k l / 16, column l % 16), result D[4i + l / 16][l % 16] in element i.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T, int GEN, int RB>
__global__ void __launch_bounds__(256) k_project_mfma(const T* Ain, double B, int nk,
                                                      long long rowsA, int wa_fixed,
                                                      const int32_t* ranks, int kin,
                                                      const double* U, T* Xout, int do_gram,
                                                      double* partials, int pstride,
                                                      int mstride) {
  constexpr int SR = 32, LT = SR + 1;
  constexpr int NCB = RB / 16;          // column blocks of Y
  constexpr int MB = 2 * RB / 16;       // blocks per side of the Gram
  constexpr int GPW = (MB * MB + 3) / 4;  // Gram blocks per wave
  extern __shared__ double smem[];
  const int WA = wa_fixed > 0 ? wa_fixed : 2 * ranks[kin - 1];
  const int r = ranks[kin];
  const int M = 2 * r;
  double* Us = smem;              // WA x r
  double* At = Us + WA * r;       // WA x LT (k-major)
  double* Ys = At + WA * LT;      // SR x r
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  for (int e = tid; e < WA * r; e += 256) Us[e] = U[e];
  f64x4 g[GPW];
#pragma unroll
  for (int t = 0; t < GPW; ++t) g[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  const long long nstage = (rowsA + SR - 1) / SR;
  // the stage's 32 x WA block, read one stage ahead into registers so that
  // its HBM latency overlaps the products of the current stage
  constexpr int PER = SR * kMaxM / 256;
  double pre[PER];
  auto fetch = [&](long long sidx) {
    const long long r0 = sidx * SR;
    const int nr = (int)((rowsA - r0) < SR ? (rowsA - r0) : SR);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = tid + 256 * j;
      const int row = e / WA, c = e - row * WA;
      pre[j] = (e < SR * WA && row < nr) ? sample<T, GEN>(Ain, (r0 + row) * WA + c, B, nk) : 0.0;
    }
  };
  if ((long long)blockIdx.x < nstage) fetch(blockIdx.x);
  for (long long sidx = blockIdx.x; sidx < nstage; sidx += gridDim.x) {
    const long long r0 = sidx * SR;
    const int nr = (int)((rowsA - r0) < SR ? (rowsA - r0) : SR);
    __syncthreads();  // At, Ys of the previous stage consumed (Us written)
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int e = tid + 256 * j;
      const int row = e / WA, c = e - row * WA;
      if (e < SR * WA) At[c * LT + row] = pre[j];
    }
    __syncthreads();
    if (sidx + gridDim.x < nstage) fetch(sidx + gridDim.x);
    // Y = A U
    {
      const int rb = w & 1;
#pragma unroll
      for (int cc = 0; cc < NCB; ++cc) {
        const int cb = (w >> 1) + 2 * cc;
        if (cb >= NCB || 16 * cb >= r) continue;  // wave-uniform
        f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
        const int col = 16 * cb + lr;
        const bool cin = col < r;
        // sixteen rows of U per pass: operands first, then four products
        for (int k16 = 0; k16 < WA; k16 += 16) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int kk = k16 + 4 * u + lk;
            const bool kin = kk < WA;
            const int kc = kin ? kk : 0;
            const double a = At[kc * LT + 16 * rb + lr];
            const double b = Us[kc * r + (cin ? col : 0)];
            av[u] = kin ? a : 0.0;
            bv[u] = (kin && cin) ? b : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * rb + 4 * i + lk;
          if (row < nr && cin) {
            Ys[row * r + col] = acc[i];
            Xout[(r0 + row) * r + col] = (T)acc[i];
          }
        }
      }
    }
    if (do_gram) {
      __syncthreads();
      // rows of Y beyond nr hold values of an earlier stage: only pairs
      // p < nr / 2 take part
      const int np = nr >> 1;
#pragma unroll
      for (int t = 0; t < GPW; ++t) {
        const int blk = w + 4 * t;
        if (blk >= MB * MB) break;
        const int bi = blk / MB, bj = blk - bi * MB;
        if (16 * bi >= M || 16 * bj >= M) continue;  // wave-uniform
        const int mi = 16 * bi + lr, nj = 16 * bj + lr;
#pragma unroll
        for (int k0 = 0; k0 < SR / 2; k0 += 4) {
          const int pk = k0 + lk;
          const bool pin = pk < np;
          const double a = (pin && mi < M) ? Ys[2 * pk * r + mi] : 0.0;
          const double bv = (pin && nj < M) ? Ys[2 * pk * r + nj] : 0.0;
          g[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, g[t], 0, 0, 0);
        }
      }
    }
  }
  if (do_gram) {
    double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
    for (int t = 0; t < GPW; ++t) {
      const int blk = w + 4 * t;
      if (blk >= MB * MB) break;
      const int bi = blk / MB, bj = blk - bi * MB;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * bi + 4 * i + lk, col = 16 * bj + lr;
        if (row < M && col < M) P[row * mstride + col] = g[t][i];
      }
    }
  }
}

// --------------------------------------------------------------- eig step
// Step k from the Gram already in A (M x M, stride lda), M = 2 r_{k-1}: the
// truncated eigendecomposition, core k, and U_k (M x r_k, row-major) in umat.
template <typename T, class MP>
__device__ int eig_step_solve(MP A, MP V, int lda, ldsd lam, ldsd sx, ldsi perm, ldsi iscr, int M,
                              int k, double tau2, int cap_k, T* cores, long long off_k,
                              double* umat, const StepOut& so) {
  constexpr int NT = kEigThreads;
  const int tid = threadIdx.x;
  const int rp = M / 2;
  const int r =
      solve_and_truncate<NT, true>(A, V, M, lda, sx, iscr, lam, perm, tau2, cap_k, k, so, true);
  for (int e = tid; e < M * r; e += NT) {
    const int c = e / r, b = e - c * r;
    umat[e] = V[c * lda + perm[b]];
  }
  const int total = rp * 2 * r;
  for (int e = tid; e < total; e += NT) {
    const int b = e % r, ai = e / r;
    const int i = ai & 1, a = ai >> 1;
    cores[off_k + e] = (T)V[(a + rp * i) * lda + perm[b]];
  }
  return r;
}

// LDS layout of an eig step: A and V in LDS for M <= kEigLds, else in gA/gV
struct EigLayout {
  double *A, *V, *lam, *sx;
  int *perm, *iscr;
  int lda;
};

__device__ __forceinline__ EigLayout eig_layout(double* smem, int M, double* gA, double* gV) {
  EigLayout L;
  if (M <= kEigLds) {
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

// eig_step_solve on a layout: A and V as LDS pointers when they live there
template <typename T>
__device__ int eig_step_solve_at(const EigLayout& L, int M, int k, double tau2, int cap_k,
                                 T* cores, long long off_k, double* umat, const StepOut& so) {
  if (M <= kEigLds)
    return eig_step_solve<T>(lds(L.A), lds(L.V), L.lda, lds(L.lam), lds(L.sx), lds(L.perm),
                             lds(L.iscr), M, k, tau2, cap_k, cores, off_k, umat, so);
  return eig_step_solve<T>(L.A, L.V, L.lda, lds(L.lam), lds(L.sx), lds(L.perm), lds(L.iscr), M,
                           k, tau2, cap_k, cores, off_k, umat, so);
}

template <typename T>
__global__ void __launch_bounds__(kEigThreads) k_eig_step(const double* gram, int mstride, int k,
                                                   const double* scal, int cap_k, T* cores,
                                                   long long off_k, double* umat,
                                                   double* gA, double* gV, StepOut so) {
  extern __shared__ double smem[];
  const int M = 2 * so.ranks[k - 1];
  const EigLayout L = eig_layout(smem, M, gA, gV);
  for (int e = threadIdx.x; e < M * M; e += kEigThreads) {
    const int i = e / M, j = e - i * M;
    L.A[i * L.lda + j] = gram[i * mstride + j];
  }
  __syncthreads();
  eig_step_solve_at<T>(L, M, k, scal[1], cap_k, cores, off_k, umat, so);
}

// -------------------------------------------------------------------- tail
// Finish the sweep from step k0 in one workgroup.  X_{k0} (n x m) comes from
// Xin (k0 > 1) or from the samples (k0 == 1, m = 2).  With k0 == 1 the norm
// and tau^2 are computed here; otherwise scal[1] holds tau^2.  gen_scale:
// divide the last core by scal[2] (generator normalisation).
template <typename T, int GEN>
__device__ void tail_steps(double* smem, const T* Xin, double B, int nk, int k0, int D,
                           double eps, const Meta& meta, T* cores, double* scal, int gen_scale,
                           const StepOut& so, int32_t* iflags) {
  constexpr int NT = kEigThreads, LDA = kEigLds + 1;
  double* X = smem;                   // kTailElems
  double* A = X + kTailElems;         // LDA*LDA  (also Y after the eigen solve)
  double* V = A + LDA * LDA;          // LDA*LDA
  double* lam = V + LDA * LDA;        // 72
  double* sx = lam + 72;              // kEigScratch
  double* red = sx + kEigScratch;     // NT
  int* perm = (int*)(red + NT);       // 72
  int* iscr = perm + 72;              // 8 + pair table (136)
  const int tid = threadIdx.x;
  int n = 1 << (D - k0);
  int rp = (k0 == 1) ? 1 : so.ranks[k0 - 1];
  int m = 2 * rp;
  double tau2;
  if (k0 == 1) {
    const long long N = 1LL << D;
    double s2 = 0.0, s1 = 0.0;
    int fin = 1;
    for (long long e = tid; e < N; e += NT) {
      const double v = sample<T, GEN>(Xin, e, B, nk);
      fin &= finite_d(v);
      X[e] = v;
      s2 += v * v;
      s1 += v;
    }
    if (!fin) atomicOr(iflags, 1);
    red[tid] = s2;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    const double nrm2 = red[0];
    __syncthreads();
    red[tid] = s1;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0) {
      scal[0] = nrm2;
      scal[2] = red[0];
      scal[1] = (D > 1) ? eps * eps * nrm2 / (double)(D - 1) : 0.0;
      so.ranks[0] = 1;
    }
    __syncthreads();
    tau2 = scal[1];
  } else {
    for (int e = tid; e < n * m; e += NT) X[e] = (double)Xin[e];
    tau2 = scal[1];
    __syncthreads();
  }
  for (int k = k0; k <= D - 1; ++k) {
#ifdef QTT_EIG_TIMING
    const long long ts0 = wall_clock64();
#endif
    const bool dual = n < m;
    const int E = dual ? n : m;
    // Gram (primal X^T X or dual X X^T)
    {
      ldsd Al = lds(A);
      auto st = [&](int i, int j, double v) { Al[i * LDA + j] = v; };
      if (!dual)
        lds_gemm_mfma(E, E, n, lds<const double>(X), 1, m, lds<const double>(X), m, 1, st);
      else
        lds_gemm_mfma(E, E, m, lds<const double>(X), m, 1, lds<const double>(X), 1, m, st);
    }
    __syncthreads();
#ifdef QTT_EIG_TIMING
    const long long ts1 = wall_clock64();
#endif
    const int r =
        solve_and_truncate<NT>(lds(A), lds(V), E, LDA, lds(sx), lds(iscr), lds(lam), lds(perm),
                               tau2, meta.caps[k], k, so, !dual);
#ifdef QTT_EIG_TIMING
    const long long ts2 = wall_clock64();
#endif
    const long long off = meta.offs[k - 1];
    const int total = rp * 2 * r;
    // U has the kept eigenvectors in its first r columns (perm is the identity)
    if (!dual) {
      for (int e = tid; e < total; e += NT) {
        const int b = e % r, ai = e / r;
        const int i = ai & 1, a = ai >> 1;
        cores[off + e] = (T)V[(a + rp * i) * LDA + b];
      }
    } else {
      // U[:, b] = X^T v_b / sigma_b
      lds_gemm_mfma(m, r, n, lds<const double>(X), 1, m, lds<const double>(V), LDA, 1,
               [&](int c, int b, double v) {
                 const double sg = lam[b] > 0.0 ? sqrt(lam[b]) : 0.0;
                 const int i = c / rp, a = c - i * rp;
                 cores[off + (long long)(a * 2 + i) * r + b] = (T)(sg > 1e-300 ? v / sg : 0.0);
               });
    }
    if (n * r <= LDA * LDA) {
      // Y (n x r, dense) into A, which the solve no longer needs
      ldsd Yl = lds(A);
      if (!dual) {
        lds_gemm_mfma(n, r, m, lds<const double>(X), m, 1, lds<const double>(V), LDA, 1,
                 [&](int row, int b, double v) { Yl[row * r + b] = v; });
      } else {
        for (int e = tid; e < n * r; e += NT) {
          const int row = e / r, b = e - row * r;
          const double sg = lam[b] > 0.0 ? sqrt(lam[b]) : 0.0;
          Yl[e] = sg * V[row * LDA + b];
        }
      }
      __syncthreads();
      // next remainder: Y (n x r) read as (n/2) x (2r)
      for (int e = tid; e < n * r; e += NT) X[e] = Yl[e];
    } else {
      // long thin remainders (few columns): Y in registers until every
      // thread has read X
      constexpr int kPer = kTailElems / NT;
      double yv[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int e = tid + j * NT;
        double sv = 0.0;
        if (e < n * r) {
          const int row = e / r, b = e - row * r;
          if (!dual) {
            for (int c = 0; c < m; ++c) sv = fma(X[row * m + c], V[c * LDA + b], sv);
          } else {
            const double sg = lam[b] > 0.0 ? sqrt(lam[b]) : 0.0;
            sv = sg * V[row * LDA + b];
          }
        }
        yv[j] = sv;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int e = tid + j * NT;
        if (e < n * r) X[e] = yv[j];
      }
    }
    __syncthreads();
#ifdef QTT_EIG_TIMING
    const long long ts3 = wall_clock64();
#endif
#ifdef QTT_EIG_TIMING
    if (tid == 0 && so.dbg) {
      const long long ts4 = wall_clock64();
      so.dbg[300 + 4 * k] = (int)(ts1 - ts0);
      so.dbg[301 + 4 * k] = (int)(ts2 - ts1);
      so.dbg[302 + 4 * k] = (int)(ts3 - ts2);
      so.dbg[303 + 4 * k] = (int)(ts4 - ts3);
    }
#endif
    n >>= 1;
    rp = r;
    m = 2 * r;
  }
  // last core (r_{D-1}, 2, 1): core[a*2 + i] = X_D[i, a] where X holds Y (2 x r)
  const double scale = (gen_scale && scal[2] != 0.0) ? 1.0 / scal[2] : 1.0;
  const long long off = meta.offs[D - 1];
  for (int e = tid; e < 2 * rp; e += NT) {
    const int a = e >> 1, i = e & 1;
    cores[off + e] = (T)(X[i * rp + a] * scale);
  }
  if (tid == 0) so.ranks[D] = 1;
}

template <typename T, int GEN>
__global__ void __launch_bounds__(kEigThreads) k_tail(const T* Xin, double B, int nk, int k0,
                                                      int D, double eps, const Meta meta,
                                                      T* cores, double* scal, int gen_scale,
                                                      StepOut so, int32_t* iflags) {
  extern __shared__ double smem[];
  tail_steps<T, GEN>(smem, Xin, B, nk, k0, D, eps, meta, cores, scal, gen_scale, so, iflags);
}

// ----------------------------------------------------------- final scaling
// Scale the last core by 1/scal[2] (used when the tail did not run the
// generator itself).
template <typename T>
__global__ void k_scale_last(T* cores, long long off, const int32_t* ranks, int D,
                             const double* scal) {
  const int rp = ranks[D - 1];
  const double s = scal[2] != 0.0 ? 1.0 / scal[2] : 1.0;
  for (int e = threadIdx.x; e < 2 * rp; e += blockDim.x) cores[off + e] = (T)((double)cores[off + e] * s);
}

// clears the per-call flag words (a kernel rather than a memset node, so
// that a captured graph replays it reliably)
__global__ void k_zero_flags(int32_t* iflags, int n) {
  if ((int)threadIdx.x < n) iflags[threadIdx.x] = 0;
}

__global__ void k_flag_status(const int32_t* iflags, int32_t* status) {
  if (threadIdx.x == 0 && status && iflags[0]) atomicOr(status, QTT_STATUS_NONFINITE);
}

// ================================================================ batched
// Many independent decompositions (lines) in one launch.  Persistent
// workgroups take the tasks (sorted by decreasing size on the host) from an
// atomic counter and run the whole sweep of a task in one workgroup, with
// the same steps as the single-signal schedule: level Gram in LDS, steps
// 1..6, projections + Grams of the remainders, eig steps, the tail.  Each
// workgroup owns a slice of global scratch (scal, U, A/V for orders > 64 and
// two remainder buffers of nmax elements).
// workgroup barrier that also orders this workgroup's global-memory writes
// (its scratch slice) before the reads that follow it; not a grid barrier
__device__ __forceinline__ void wg_barrier_with_global_fence() {
  __threadfence();
  __syncthreads();
}

template <typename T, int GEN, int TS>
__device__ __noinline__ void batch_project(const T* Ain, double B, int nk, long long rowsA, int WA, int r,
                              const double* U, T* Xout, int do_gram, ldsd smem_l, int M,
                              const EigLayout& Ly) {
  // generic view of the LDS pointer: its accesses still compile to ds_*
  double* smem = (double*)smem_l;
  double acc[TS][TS];
  project_gram_acc<T, GEN, TS>(Ain, B, nk, rowsA, WA, r, U, Xout, do_gram, 0, 1, smem, acc);
  if (do_gram) {
    // the projection's LDS is free after its last barrier; A may overlap it
    const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
#pragma unroll
    for (int a = 0; a < TS; ++a)
#pragma unroll
      for (int c = 0; c < TS; ++c) {
        const int i = ty * TS + a, j = tx * TS + c;
        if (i < M && j < M) Ly.A[i * Ly.lda + j] = acc[a][c];
      }
  }
  wg_barrier_with_global_fence();
}

template <typename T, int GEN>
__device__ void batch_project_any(int Mcap, const T* Ain, double B, int nk, long long rowsA,
                                  int WA, int r, const double* U, T* Xout, int do_gram,
                                  double* smem, int M, const EigLayout& Ly) {
  if (Mcap <= 16)
    batch_project<T, GEN, 1>(Ain, B, nk, rowsA, WA, r, U, Xout, do_gram, lds(smem), M, Ly);
  else if (Mcap <= 32)
    batch_project<T, GEN, 2>(Ain, B, nk, rowsA, WA, r, U, Xout, do_gram, lds(smem), M, Ly);
  else if (Mcap <= 64)
    batch_project<T, GEN, 4>(Ain, B, nk, rowsA, WA, r, U, Xout, do_gram, lds(smem), M, Ly);
  else
    batch_project<T, GEN, 8>(Ain, B, nk, rowsA, WA, r, U, Xout, do_gram, lds(smem), M, Ly);
}

template <typename T, int GEN>
__device__ __noinline__ void batch_line(const BatchTask& tk, const T* x, T* cores, int32_t* ranks,
                           int32_t* status, ldsd smem_l, Meta& meta, double* wscr, T* xb0,
                           T* xb1) {
  double* smem = (double*)smem_l;  // LDS (accesses compile to ds_*)
  const int tid = threadIdx.x;
  const int D = tk.D;
  double* scal = wscr;
  double* umat = scal + 16;
  double* gA = umat + kMaxM * kMaxRank;
  double* gV = gA + (kMaxM + 1) * (kMaxM + 1);
  // capacities and (absolute) core offsets of this task
  if (tid == 0) {
    long long off = tk.core_off;
    for (int k = 0; k <= D; ++k) {
      int c = tk.rcap;
      if (k < 30 && (1 << k) < c) c = 1 << k;
      if (D - k < 30 && (1 << (D - k)) < c) c = 1 << (D - k);
      meta.caps[k] = (k == 0 || k == D) ? 1 : c;
    }
    for (int k = 0; k < D; ++k) {
      meta.offs[k] = off;
      const int c1 = (k + 1 == D) ? 1 : meta.caps[k + 1];
      off += (long long)meta.caps[k] * 2 * c1;
    }
    meta.offs[D] = off;
  }
  __syncthreads();
  StepOut so;
  so.ranks = ranks + tk.rank_off;
  so.status = status + tk.status_idx;
  so.sv = nullptr;
  so.lib_capped = tk.rcap >= kMaxRank ? 1 : 0;
  so.dbg = nullptr;
  so.delta2 = 0.0;
  int32_t* flag = status + tk.status_idx;  // non-finite input sets bit 1 here directly
  const T* xl = GEN ? x : x + tk.x_off;
  const long long N = 1LL << D;
  if (D == 1) {
    if (tid == 0) {
      const double v0 = sample<T, GEN>(xl, 0, tk.B, tk.nk), v1 = sample<T, GEN>(xl, 1, tk.B, tk.nk);
      double sm = (GEN == 1) ? v0 + v1 : 1.0;
      if (sm == 0.0) sm = 1.0;
      cores[meta.offs[0]] = (T)(v0 / sm);
      cores[meta.offs[0] + 1] = (T)(v1 / sm);
      so.ranks[0] = 1;
      so.ranks[1] = 1;
      if (!(finite_d(v0) && finite_d(v1))) atomicOr(flag, QTT_STATUS_NONFINITE);
    }
    return;
  }
  if (N <= kTailElems) {
    tail_steps<T, GEN>(smem, xl, tk.B, tk.nk, 1, D, tk.eps, meta, cores, scal, GEN == 1, so, flag);
    return;
  }
  // level Gram of the samples viewed as (N/64) x 64, straight into LDS
  const int L = kLevel;
  {
    double acc[4][4];
    double gsum;
    int fin;
    level_gram_acc<T, GEN>(xl, tk.B, tk.nk, N >> L, 0, 1, smem, acc, gsum, fin);
    const double tot = wg_sum256(gsum, smem + 64 * 64);
    const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) smem[(4 * ty + a) * 64 + 4 * tx + b] = acc[a][b];
    if (!fin) atomicOr(flag, QTT_STATUS_NONFINITE);
    if (tid == 0) scal[2] = tot;
    __syncthreads();
  }
  level_steps<T>(smem, L, D, tk.eps, meta, cores, scal, umat, so);
  wg_barrier_with_global_fence();
  int tail_k = L + 1;
  while (tail_k < D && !((1LL << (D - tail_k)) * 2LL * meta.caps[tail_k - 1] <= kTailElems))
    ++tail_k;
  int k = L + 1;
  T* xb[2] = {xb0, xb1};
  int cur = 0;
  {
    const int r = so.ranks[L];
    const int M = 2 * r;
    const EigLayout Ly = eig_layout(smem, M, gA, gV);
    batch_project_any<T, GEN>(2 * meta.caps[L], xl, tk.B, tk.nk, N >> L, 1 << L, r, umat, xb[cur],
                              k < tail_k ? 1 : 0, smem, M, Ly);
  }
  while (k < tail_k) {
    const int rp = so.ranks[k - 1];
    const int M = 2 * rp;
    const EigLayout Ly = eig_layout(smem, M, gA, gV);
    const int r = eig_step_solve_at<T>(Ly, M, k, scal[1], meta.caps[k], cores, meta.offs[k - 1],
                                       umat, so);
    wg_barrier_with_global_fence();
    const int M2 = 2 * r;
    const EigLayout Ly2 = eig_layout(smem, M2, gA, gV);
    batch_project_any<T, 0>(2 * meta.caps[k], xb[cur], tk.B, tk.nk, 1LL << (D - k), M, r, umat,
                            xb[cur ^ 1], (k + 1 < tail_k) ? 1 : 0, smem, M2, Ly2);
    cur ^= 1;
    ++k;
  }
  tail_steps<T, 0>(smem, xb[cur], tk.B, tk.nk, k, D, tk.eps, meta, cores, scal, 0, so, flag);
  if (GEN == 1) {
    wg_barrier_with_global_fence();
    const int rp = so.ranks[D - 1];
    const double sc = scal[2] != 0.0 ? 1.0 / scal[2] : 1.0;
    T* last = cores + meta.offs[D - 1];
    for (int e = tid; e < 2 * rp; e += kEigThreads) last[e] = (T)((double)last[e] * sc);
  }
}

template <typename T, int GEN>
__global__ void __launch_bounds__(kEigThreads) k_batch_decompose(
    const T* x, const BatchTask* tasks, int ntasks, int32_t* counter, T* cores, int32_t* ranks,
    int32_t* status, char* wscr, long long wstride, long long nmax) {
  extern __shared__ double smem[];
  __shared__ int s_task;
  __shared__ Meta s_meta;
  double* my = reinterpret_cast<double*>(wscr + (long long)blockIdx.x * wstride);
  T* xb0 = reinterpret_cast<T*>(my + batch_wg_doubles());
  T* xb1 = xb0 + nmax;
  for (;;) {
    if (threadIdx.x == 0) s_task = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_task;
    __syncthreads();
    if (t >= ntasks) break;  // every wave leaves on the same value
    const BatchTask tk = tasks[t];
    batch_line<T, GEN>(tk, x, cores, ranks, status, lds(smem), s_meta, my, xb0, xb1);
    wg_barrier_with_global_fence();
  }
}

// =================================================================== host
static size_t lds_level_eig() {
  return sizeof(double) * (64 * 64 + 2 * 65 * 65 + 64 * 64 + 32 * 32 + 72 + kEigScratch) +
         sizeof(int) * (72 + 8 + 256);
}
static size_t lds_eig_step() {
  const int lda = kEigLds + 1;
  return sizeof(double) * (2 * lda * lda + (kMaxM + 8) + kEigScratch) +
         sizeof(int) * (kMaxM + 8 + 8 + 256);
}
static size_t lds_tail() {
  const int lda = kEigLds + 1;
  return sizeof(double) * (kTailElems + 2 * lda * lda + 72 + kEigScratch + kEigThreads) +
         sizeof(int) * (72 + 8 + 256);
}
static size_t lds_project(int wa, int r) {
  return sizeof(double) * ((size_t)wa * r + 32 * (size_t)wa + 32 * (size_t)r);
}
static size_t lds_project_mfma(int wa, int r) {
  return sizeof(double) * ((size_t)wa * r + 33 * (size_t)wa + 32 * (size_t)r);
}

int plan_decompose(int D, int rcap, int dtype, void* ws, DecompPlan* p) {
  DecompPlan& P = *p;
  P.D = D;
  P.dtype = dtype;
  P.rcap = rcap;
  for (int k = 0; k <= D; ++k) {
    int c = rcap;
    const int lo = k < 30 ? (1 << k) : (1 << 30);
    const int hi = (D - k) < 30 ? (1 << (D - k)) : (1 << 30);
    if (lo < c) c = lo;
    if (hi < c) c = hi;
    P.cap[k] = (k == 0 || k == D) ? 1 : c;
  }
  const long long N = 1LL << D;
  P.use_level = (D > 1 && N > kTailElems) ? 1 : 0;
  // first tail step
  P.tail_k = 1;
  if (P.use_level) {
    int k = kLevel + 1;
    while (k < D && !((1LL << (D - k)) * 2LL * P.cap[k - 1] <= kTailElems)) ++k;
    P.tail_k = k;
  }
  int mcap = 2;
  for (int k = 1; k < D; ++k) mcap = mcap > 2 * P.cap[k - 1] ? mcap : 2 * P.cap[k - 1];
  if (mcap < 64) mcap = 64;
  P.gstride = mcap;
  P.pstride = mcap * mcap;
  Arena ar(ws);
  P.scal = ar.take<double>(16);
  // [0] non-finite flag, [16+k] Gram order of step k, [80+5k..] optional timings
  P.iflags = ar.take<int32_t>(16 + 64 + 512);
  P.gram = ar.take<double>((size_t)mcap * mcap);
  P.umat = ar.take<double>((size_t)kMaxM * kMaxRank);
  P.gpart_sum = ar.take<double>(kMaxPartials);
  if (P.use_level) {
    P.partials = ar.take<double>((size_t)kMaxPartials * P.pstride);
    P.eigA = ar.take<double>((size_t)(kMaxM + 1) * (kMaxM + 1));
    P.eigV = ar.take<double>((size_t)(kMaxM + 1) * (kMaxM + 1));
    const size_t es = elem_size(dtype);
    char* b0 = ar.take<char>((size_t)N * es);
    char* b1 = ar.take<char>((size_t)N * es);
    P.xbuf[0] = b0;
    P.xbuf[1] = b1;
  } else {
    P.partials = nullptr;
    P.eigA = P.eigV = nullptr;
    P.xbuf[0] = P.xbuf[1] = nullptr;
  }
  P.ws_bytes = ar.size();
  return QTT_OK;
}

template <typename T, int GEN>
static hipError_t set_attrs() {
  hipError_t e = hipSuccess;
  set_lds_limit((const void*)k_level_eig<T>, (int)lds_level_eig(), &e);
  set_lds_limit((const void*)k_eig_step<T>, (int)lds_eig_step(), &e);
  set_lds_limit((const void*)k_tail<T, 0>, (int)lds_tail(), &e);
  set_lds_limit((const void*)k_tail<T, 1>, (int)lds_tail(), &e);
  set_lds_limit((const void*)k_tail<T, GEN>, (int)lds_tail(), &e);
  set_lds_limit((const void*)k_project_gram<T, GEN, 1>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, GEN, 2>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, GEN, 4>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, GEN, 8>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, 0, 1>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, 0, 2>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, 0, 4>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_gram<T, 0, 8>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_mfma<T, GEN, 16>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_mfma<T, GEN, 32>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_mfma<T, GEN, 64>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_mfma<T, 0, 16>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_mfma<T, 0, 32>, 160 * 1024, &e);
  set_lds_limit((const void*)k_project_mfma<T, 0, 64>, 160 * 1024, &e);
  return e;
}

template <typename T, int GEN>
static int launch_project(const T* Ain, const Source& src, long long rowsA, int wa_fixed,
                          int wa_cap, const int32_t* ranks, int kin, int rcap_out,
                          const double* U, T* Xout, int do_gram, const DecompPlan& P,
                          int mstride, int* nparts, hipStream_t stream) {
  constexpr int SR = 32;
  long long nstage = (rowsA + SR - 1) / SR;
  int blocks = (int)(nstage < kMaxPartials ? nstage : kMaxPartials);
  if (blocks < 1) blocks = 1;
  *nparts = blocks;
  const int Mc = 2 * rcap_out;
  ProbeScope _ps(QTT_K_PROJECT, stream);
  if (rcap_out <= kMaxRank) {
    const size_t lm = lds_project_mfma(wa_cap, rcap_out);
    if (rcap_out <= 16)
      k_project_mfma<T, GEN, 16><<<blocks, 256, lm, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                              ranks, kin, U, Xout, do_gram,
                                                              P.partials, P.pstride, mstride);
    else if (rcap_out <= 32)
      k_project_mfma<T, GEN, 32><<<blocks, 256, lm, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                              ranks, kin, U, Xout, do_gram,
                                                              P.partials, P.pstride, mstride);
    else
      k_project_mfma<T, GEN, 64><<<blocks, 256, lm, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                              ranks, kin, U, Xout, do_gram,
                                                              P.partials, P.pstride, mstride);
    QTT_LAUNCH_CHECK();
    return QTT_OK;
  }
  const size_t lds = lds_project(wa_cap, rcap_out);
  if (Mc <= 16) {
    k_project_gram<T, GEN, 1><<<blocks, 256, lds, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                            ranks, kin, U, Xout, do_gram,
                                                            P.partials, P.pstride, mstride);
  } else if (Mc <= 32) {
    k_project_gram<T, GEN, 2><<<blocks, 256, lds, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                            ranks, kin, U, Xout, do_gram,
                                                            P.partials, P.pstride, mstride);
  } else if (Mc <= 64) {
    k_project_gram<T, GEN, 4><<<blocks, 256, lds, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                            ranks, kin, U, Xout, do_gram,
                                                            P.partials, P.pstride, mstride);
  } else {
    k_project_gram<T, GEN, 8><<<blocks, 256, lds, stream>>>(Ain, src.B, src.nk, rowsA, wa_fixed,
                                                            ranks, kin, U, Xout, do_gram,
                                                            P.partials, P.pstride, mstride);
  }
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

template <typename T, int GEN>
static int run_decompose_t(const DecompPlan& P, const Source& src, double eps,
                           const TensorDev& out, double* sv, hipStream_t stream, double delta) {
  // kernel attributes once per instantiation, safe under concurrent first calls
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] { attr_err = set_attrs<T, GEN>(); });
  QTT_HIP_CHECK(attr_err);
  const int D = P.D;
  const T* x = static_cast<const T*>(src.x);
  T* cores = static_cast<T*>(out.cores);
  StepOut so;
  so.ranks = out.ranks;
  so.status = out.status;
  so.sv = sv;
  so.lib_capped = P.rcap >= kMaxRank ? 1 : 0;
  so.dbg = P.iflags + 16;
  so.delta2 = delta * delta;
  Meta meta;
  for (int k = 0; k <= QTT_MAXD; ++k) {
    meta.caps[k] = k <= D ? P.cap[k] : 0;
    meta.offs[k] = k <= D ? out.off[k] : 0;
  }
  {
    ProbeScope _ps(QTT_K_OTHER, stream);
    k_zero_flags<<<1, 64, 0, stream>>>(P.iflags, 16);
  }
  QTT_LAUNCH_CHECK();
  if (D == 1) {
    {
      ProbeScope _ps(QTT_K_OTHER, stream);
      k_single<T, GEN><<<1, 64, 0, stream>>>(x, src.B, src.nk, cores, out.ranks, P.scal, out.status);
    }
    QTT_LAUNCH_CHECK();
    return QTT_OK;
  }
  if (!P.use_level) {
    {
      ProbeScope _ps(QTT_K_TAIL, stream);
      k_tail<T, GEN><<<1, kEigThreads, lds_tail(), stream>>>(x, src.B, src.nk, 1, D, eps, meta, cores,
                                                     P.scal, src.gen == 1, so, P.iflags);
    }
    QTT_LAUNCH_CHECK();
    {
      ProbeScope _ps(QTT_K_OTHER, stream);
      k_flag_status<<<1, 64, 0, stream>>>(P.iflags, out.status);
    }
    QTT_LAUNCH_CHECK();
    return QTT_OK;
  }
  const long long N = 1LL << D;
  const int L = kLevel;
  // 1. Gram of the samples viewed as (N/64) x 64
  {
    const long long rows = N >> L;
    long long nstage = (rows + 31) / 32;
    int blocks = (int)(nstage < kMaxPartials ? nstage : kMaxPartials);
    {
      ProbeScope _ps(QTT_K_LEVEL_GRAM, stream);
      k_level_gram<T, GEN><<<blocks, 256, 0, stream>>>(x, src.B, src.nk, rows, P.partials, P.pstride,
                                                     P.gpart_sum, P.iflags);
    }
    QTT_LAUNCH_CHECK();
    {
      ProbeScope _ps(QTT_K_REDUCE, stream);
      k_reduce<<<(64 * 64 + 63) / 64, 256, 0, stream>>>(P.partials, P.pstride, blocks, 64 * 64,
                                                         P.gram, P.gpart_sum, P.scal);
    }
    QTT_LAUNCH_CHECK();
  }
  // 2. steps 1..L
  {
    ProbeScope _ps(QTT_K_LEVEL_EIG, stream);
    k_level_eig<T><<<1, kEigThreads, lds_level_eig(), stream>>>(P.gram, L, D, eps, meta, cores, P.scal,
                                                       P.umat, so);
  }
  QTT_LAUNCH_CHECK();
  // 3. X_{L+1} = Z_L Phi_L, Gram of X_{L+1}
  int cur = 0;
  int k = L + 1;
  int nparts = 0;
  {
    const bool tail_now = (k >= P.tail_k);
    const int mstride = 2 * P.cap[L];
    int rc = launch_project<T, GEN>(x, src, N >> L, 1 << L, 1 << L, out.ranks, L, P.cap[L],
                                    P.umat, static_cast<T*>(P.xbuf[cur]), tail_now ? 0 : 1, P,
                                    mstride, &nparts, stream);
    if (rc) return rc;
  }
  while (k < P.tail_k) {
    // Gram of X_k is in the partials (stride 2 cap_{k-1})
    const int mstride = 2 * P.cap[k - 1];
    {
      ProbeScope _ps(QTT_K_REDUCE, stream);
      k_reduce<<<(mstride * mstride + 63) / 64, 256, 0, stream>>>(
        P.partials, P.pstride, nparts, mstride * mstride, P.gram, nullptr, nullptr, out.ranks, k,
        mstride);
    }
    QTT_LAUNCH_CHECK();
    {
      ProbeScope _ps(QTT_K_EIG_STEP, stream);
      k_eig_step<T><<<1, kEigThreads, lds_eig_step(), stream>>>(P.gram, mstride, k, P.scal, P.cap[k], cores,
                                                       out.off[k - 1], P.umat, P.eigA, P.eigV, so);
    }
    QTT_LAUNCH_CHECK();
    // X_{k+1} = X_k U_k
    const long long rowsA = 1LL << (D - k);
    const bool tail_next = (k + 1 >= P.tail_k);
    const int mnext = 2 * P.cap[k];
    int rc = launch_project<T, 0>(static_cast<const T*>(P.xbuf[cur]), src, rowsA, 0,
                                  2 * P.cap[k - 1], out.ranks, k, P.cap[k], P.umat,
                                  static_cast<T*>(P.xbuf[cur ^ 1]), tail_next ? 0 : 1, P, mnext,
                                  &nparts, stream);
    if (rc) return rc;
    cur ^= 1;
    ++k;
  }
  {
    ProbeScope _ps(QTT_K_TAIL, stream);
    k_tail<T, 0><<<1, kEigThreads, lds_tail(), stream>>>(static_cast<const T*>(P.xbuf[cur]), src.B,
                                                src.nk, k, D, eps, meta, cores, P.scal, 0, so,
                                                P.iflags);
  }
  QTT_LAUNCH_CHECK();
  if (src.gen == 1) {
    {
      ProbeScope _ps(QTT_K_OTHER, stream);
      k_scale_last<T><<<1, 256, 0, stream>>>(cores, out.off[D - 1], out.ranks, D, P.scal);
    }
    QTT_LAUNCH_CHECK();
  }
  {
    ProbeScope _ps(QTT_K_OTHER, stream);
    k_flag_status<<<1, 64, 0, stream>>>(P.iflags, out.status);
  }
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_decompose(const DecompPlan& P, const Source& src, double eps, const TensorDev& out,
                  double* sv, hipStream_t stream, double delta) {
  if (P.dtype == QTT_F64) {
    if (src.gen == 2) return run_decompose_t<double, 2>(P, src, eps, out, sv, stream, delta);
    return src.gen ? run_decompose_t<double, 1>(P, src, eps, out, sv, stream, delta)
                   : run_decompose_t<double, 0>(P, src, eps, out, sv, stream, delta);
  }
  if (src.gen == 2) return run_decompose_t<float, 2>(P, src, eps, out, sv, stream, delta);
  return src.gen ? run_decompose_t<float, 1>(P, src, eps, out, sv, stream, delta)
                 : run_decompose_t<float, 0>(P, src, eps, out, sv, stream, delta);
}

}  // namespace qtt

// ------------------------------------------------------------ batched host
namespace qtt {

size_t batch_decompose_lds() {
  size_t m = lds_level_eig();
  if (lds_tail() > m) m = lds_tail();
  if (lds_eig_step() > m) m = lds_eig_step();
  const size_t pj = lds_project(kMaxM, kMaxRank);
  if (pj > m) m = pj;
  return m;
}

template <typename T, int GEN>
static int batch_decompose_t(const T* x, const BatchTask* tasks, int ntasks, int32_t* counter,
                             T* cores, int32_t* ranks, int32_t* status, char* wscr,
                             long long wstride, long long nmax, int nwg, hipStream_t s) {
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] {
    set_lds_limit((const void*)k_batch_decompose<T, GEN>, (int)batch_decompose_lds(), &attr_err);
  });
  QTT_HIP_CHECK(attr_err);
  ProbeScope _ps(QTT_K_BATCH, s);
  k_batch_decompose<T, GEN><<<nwg, kEigThreads, batch_decompose_lds(), s>>>(
      x, tasks, ntasks, counter, cores, ranks, status, wscr, wstride, nmax);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_batch_decompose(int dtype, int gen, const void* x, const BatchTask* tasks, int ntasks,
                        int32_t* counter, void* cores, int32_t* ranks, int32_t* status,
                        char* wscr, long long wstride, long long nmax, int nwg, hipStream_t s) {
  if (dtype == QTT_F64) {
    if (gen)
      return batch_decompose_t<double, 1>(static_cast<const double*>(x), tasks, ntasks, counter,
                                          static_cast<double*>(cores), ranks, status, wscr,
                                          wstride, nmax, nwg, s);
    return batch_decompose_t<double, 0>(static_cast<const double*>(x), tasks, ntasks, counter,
                                        static_cast<double*>(cores), ranks, status, wscr, wstride,
                                        nmax, nwg, s);
  }
  if (gen)
    return batch_decompose_t<float, 1>(static_cast<const float*>(x), tasks, ntasks, counter,
                                       static_cast<float*>(cores), ranks, status, wscr, wstride,
                                       nmax, nwg, s);
  return batch_decompose_t<float, 0>(static_cast<const float*>(x), tasks, ntasks, counter,
                                     static_cast<float*>(cores), ranks, status, wscr, wstride,
                                     nmax, nwg, s);
}

}  // namespace qtt

// Randomised rounding (the precision form): the TT-SVD sweep of a full
// vector in which every truncated SVD is taken by the randomised range
// finder and RSVD (Algorithms 4 and 5, Appendix A).
//
// Step k works on the remainder X_k (n x m row-major, m = 2 r_{k-1}; the
// unfolding is A = X_k^T).  When the sketch is narrower than the unfolding
// (ell < m):
//   1. one streaming pass forms Y = A Omega (m x ell) on the matrix cores --
//      bfloat16 operands (v_mfma_f32_16x16x32_bf16) or single-precision
//      operands (v_mfma_f32_16x16x4f32), FP32 accumulation, FP64 combine of
//      the per-block partials; Omega is drawn in the kernel;
//   2. one workgroup: Q = qr(Y) (FP64 Householder);
//   3. a second pass forms B = Q^T A per tile and accumulates B B^T, both on
//      the FP32 matrix cores with single-precision operands;
//   4. one workgroup: the eigendecomposition of B B^T gives sigma(B) and U~,
//      the rank rule of Algorithm 1 picks r, U = Q U~_r is core k;
//   5. X_{k+1} = X_k U read as (n/2) x 2r (the remainder U^T A).
// No Gram of A is formed on such steps.  With ell >= m the range finder spans
// all of R^m and the step is the exact SVD: one pass forms the FP64 Gram and
// the step takes its eigendecomposition.
// Omega[row][col] of step k is one standard normal from Philox-4x32-10 with
// counter (row, col, k, 0) and key (seed low, seed high) through the
// Box-Muller transform of its first two words.
#include <math.h>

#include <mutex>

#include "qtt_eig.hpp"
#include "qtt_internal.hpp"
#include "qtt_philox.hpp"

namespace qtt {

// ----------------------------------------------------------- exact steps
// Partials of the FP64 Gram G = A A^T per block (row stride pstride), for
// steps whose sketch covers the unfolding (m <= ell); no-op otherwise.
// Thread (ty, tx) owns the TS x TS tile of G at rows ty*TS.., cols tx*TS...
constexpr int kSkSR = 32;
constexpr int kSkMaxEll = 64;

template <typename T, int TS>
__global__ void __launch_bounds__(256) k_gram_sketch(const T* X, long long n, const int32_t* ranks,
                                                     int kin, int ell, double* partials,
                                                     int pstride) {
  extern __shared__ double smem[];
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  if (m > ell) return;  // a sketched step (uniform)
  double* Xs = smem;    // kSkSR x m
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  double g[TS][TS];
#pragma unroll
  for (int a = 0; a < TS; ++a)
#pragma unroll
    for (int b = 0; b < TS; ++b) g[a][b] = 0.0;
  const long long nstage = (n + kSkSR - 1) / kSkSR;
  for (long long sidx = blockIdx.x; sidx < nstage; sidx += gridDim.x) {
    const long long r0 = sidx * kSkSR;
    const int nr = (int)((n - r0) < kSkSR ? (n - r0) : kSkSR);
    for (int e = tid; e < kSkSR * m; e += 256) Xs[e] = (e / m < nr) ? (double)X[r0 * m + e] : 0.0;
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const double* xr = Xs + rr * m;
      double xa[TS], xb[TS];
#pragma unroll
      for (int a = 0; a < TS; ++a) {
        const int i = ty * TS + a;
        xa[a] = i < m ? xr[i] : 0.0;
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
  }
}

// ---------------------------------------------- sketch GEMMs, matrix cores
// Operand formats: BF = 1 rounds every operand to bfloat16 (round to
// nearest, ties to even, from its single-precision value) and multiplies on
// v_mfma_f32_16x16x32_bf16; BF = 0 multiplies single-precision operands on
// v_mfma_f32_16x16x4f32.  Both accumulate in FP32.  The lane layouts (one
// 16 x 16 output block per instruction, D[4 (l / 16) + e][l % 16] in
// accumulator e):
//   16x16x32 bf16: lane l holds A[l % 16][8 (l / 16) + 0..7] and
//                  B[8 (l / 16) + 0..7][l % 16];
//   16x16x4 f32:   lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
typedef float sk_f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 sk_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short sk_u16x8 __attribute__((ext_vector_type(8)));

// bfloat16 bits of x (round to nearest, ties to even; x finite)
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// the operand element type of the LDS tiles
template <int BF>
struct SkOp;
template <>
struct SkOp<1> {
  using T = unsigned short;
  static __device__ __forceinline__ unsigned short cvt(double x) { return bf16_bits((float)x); }
};
template <>
struct SkOp<0> {
  using T = float;
  static __device__ __forceinline__ float cvt(double x) { return (float)x; }
};

// acc += the 16 x 16 product of a 16 x KB panel of Pa (rows ra0.., row
// stride lda, k contiguous) and a KB x 16 panel given by its transpose Pb
// (rows rb0.., row stride ldb, k contiguous); KB a multiple of 32 (bfloat16)
// or 4 (single precision)
template <int BF>
__device__ __forceinline__ sk_f32x4 sk_panel(const typename SkOp<BF>::T* Pa, int lda, int ra0,
                                             const typename SkOp<BF>::T* Pb, int ldb, int rb0,
                                             int KB, sk_f32x4 acc) {
  const int l = threadIdx.x & 63;
  if constexpr (BF == 1) {
    for (int k0 = 0; k0 < KB; k0 += 32) {
      const sk_u16x8 ua =
          *reinterpret_cast<const sk_u16x8*>(Pa + (ra0 + (l & 15)) * lda + k0 + 8 * (l >> 4));
      const sk_u16x8 ub =
          *reinterpret_cast<const sk_u16x8*>(Pb + (rb0 + (l & 15)) * ldb + k0 + 8 * (l >> 4));
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(sk_bf16x8, ua),
                                                    __builtin_bit_cast(sk_bf16x8, ub), acc, 0, 0,
                                                    0);
    }
  } else {
    for (int k0 = 0; k0 < KB; k0 += 4) {
      const float fa = Pa[(ra0 + (l & 15)) * lda + k0 + (l >> 4)];
      const float fb = Pb[(rb0 + (l & 15)) * ldb + k0 + (l >> 4)];
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, fb, acc, 0, 0, 0);
    }
  }
  return acc;
}

// Partials of Y = A Omega (m x ell) per block, for m > ell (no-op otherwise).
// A stage of kSkSR rows of X gives the transposed tiles Xt[i][rr] = X[rr][i]
// (m_pad x kSkSR) and Ot[c][rr] = Omega[rr][c] (ell_pad x kSkSR); wave w
// accumulates the output blocks w, w + 4, ... of the (m/16) x (ell/16) grid.
constexpr int kSkLd = kSkSR + 8;  // LDS row stride of the stage tiles (elements)

template <typename T, int BF>
__global__ void __launch_bounds__(256) k_sketch_y(const T* X, long long n, const int32_t* ranks,
                                                  int kin, int ell, uint32_t key0, uint32_t key1,
                                                  int step, double* partials, int pstride) {
  using OT = typename SkOp<BF>::T;
  extern __shared__ double smem[];
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  if (m <= ell) return;  // the step is exact (uniform)
  const int mp = (m + 15) & ~15, ep = (ell + 15) & ~15;
  OT* Xt = reinterpret_cast<OT*>(smem);  // mp x kSkLd
  OT* Ot = Xt + mp * kSkLd;               // ep x kSkLd
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int nbi = mp / 16, nbj = ep / 16, nb = nbi * nbj;
  sk_f32x4 acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = sk_f32x4{0.f, 0.f, 0.f, 0.f};
  const long long nstage = (n + kSkSR - 1) / kSkSR;
  for (long long sidx = blockIdx.x; sidx < nstage; sidx += gridDim.x) {
    const long long r0 = sidx * kSkSR;
    const int nr = (int)((n - r0) < kSkSR ? (n - r0) : kSkSR);
    for (int e = tid; e < kSkSR * mp; e += 256) {
      const int rr = e / mp, i = e - rr * mp;
      const double v = (rr < nr && i < m) ? (double)X[(r0 + rr) * m + i] : 0.0;
      Xt[i * kSkLd + rr] = SkOp<BF>::cvt(v);
    }
    for (int e = tid; e < kSkSR * ep; e += 256) {
      const int rr = e / ep, c = e - rr * ep;
      const double v = (rr < nr && c < ell) ? omega_entry(r0 + rr, c, step, key0, key1) : 0.0;
      Ot[c * kSkLd + rr] = SkOp<BF>::cvt(v);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int b = w + 4 * t;
      if (b < nb) {
        const int bi = b / nbj, bj = b - bi * nbj;
        acc[t] = sk_panel<BF>(Xt, kSkLd, 16 * bi, Ot, kSkLd, 16 * bj, kSkSR, acc[t]);
      }
    }
    __syncthreads();
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int b = w + 4 * t;
    if (b >= nb) continue;
    const int bi = b / nbj, bj = b - bi * nbj;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * bi + 4 * (l >> 4) + e, c = 16 * bj + (l & 15);
      if (i < m && c < ell) P[i * ell + c] = (double)acc[t][e];
    }
  }
}

// Partials of G_B = B B^T (ell x ell) with B = Q^T A, for m > ell (no-op
// otherwise).  Q^T (ell x m) sits in LDS for the whole pass (Qt[c][i]); a
// stage of kSkSR rows of X (Xs[rr][i], rows of X are columns of A) gives the
// tile B_s = Q^T A_s (ell x kSkSR), then B_s B_s^T is accumulated; both on
// the FP32 matrix cores with single-precision operands (for either operand
// format of the sketch: B decides the singular values and the kept basis).
template <typename T>
__global__ void __launch_bounds__(256) k_sketch_gb(const T* X, long long n, const int32_t* ranks,
                                                   int kin, int ell, const double* Q,
                                                   double* partials, int pstride) {
  constexpr int BF = 0;
  using OT = typename SkOp<BF>::T;
  extern __shared__ double smem[];
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  if (m <= ell) return;
  const int mk = (m + 31) & ~31, ep = (ell + 15) & ~15;
  const int ldq = mk + 8;
  OT* Qt = reinterpret_cast<OT*>(smem);  // ep x ldq
  OT* Xs = Qt + ep * ldq;                 // kSkSR x ldq
  float* Bt = reinterpret_cast<float*>(Xs + kSkSR * ldq);  // ep x (kSkSR + 4)
  constexpr int ldb = kSkSR + 4;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int e = tid; e < ep * mk; e += 256) {
    const int c = e / mk, i = e - c * mk;
    Qt[c * ldq + i] = SkOp<BF>::cvt((c < ell && i < m) ? Q[i * ell + c] : 0.0);
  }
  const int nbe = ep / 16;
  const int nbs = nbe * (kSkSR / 16);  // blocks of the stage product B_s
  const int nbg = nbe * nbe;           // blocks of G_B
  sk_f32x4 g[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) g[t] = sk_f32x4{0.f, 0.f, 0.f, 0.f};
  const long long nstage = (n + kSkSR - 1) / kSkSR;
  for (long long sidx = blockIdx.x; sidx < nstage; sidx += gridDim.x) {
    const long long r0 = sidx * kSkSR;
    const int nr = (int)((n - r0) < kSkSR ? (n - r0) : kSkSR);
    for (int e = tid; e < kSkSR * mk; e += 256) {
      const int rr = e / mk, i = e - rr * mk;
      const double v = (rr < nr && i < m) ? (double)X[(r0 + rr) * m + i] : 0.0;
      Xs[rr * ldq + i] = SkOp<BF>::cvt(v);
    }
    __syncthreads();
    // B_s blocks: wave w takes w, w + 4 (at most 8 blocks: ell <= 64, 2 column blocks)
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int b = w + 4 * t;
      if (b < nbs) {
        const int bi = b >> 1, bj = b & 1;
        sk_f32x4 acc = sk_f32x4{0.f, 0.f, 0.f, 0.f};
        acc = sk_panel<BF>(Qt, ldq, 16 * bi, Xs, ldq, 16 * bj, mk, acc);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          Bt[(16 * bi + 4 * (l >> 4) + e) * ldb + 16 * bj + (l & 15)] = acc[e];
      }
    }
    __syncthreads();
    // G_B += B_s B_s^T: wave w takes the blocks w, w + 4, ... of (ell/16)^2
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int b = w + 4 * t;
      if (b < nbg) {
        const int bi = b / nbe, bj = b - bi * nbe;
        g[t] = sk_panel<0>(Bt, ldb, 16 * bi, Bt, ldb, 16 * bj, kSkSR, g[t]);
      }
    }
    __syncthreads();
  }
  double* P = partials + (size_t)blockIdx.x * pstride;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int b = w + 4 * t;
    if (b >= nbg) continue;
    const int bi = b / nbe, bj = b - bi * nbe;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * bi + 4 * (l >> 4) + e, c = 16 * bj + (l & 15);
      if (i < ell && c < ell) P[i * ell + c] = (double)g[t][e];
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

// out[e] = sum over the partials of entry e (fixed order).  what: 0 the Gram
// of an exact step (m x m, only when m <= ell), 1 the sketch Y (m x ell) and
// 2 the matrix B B^T (ell x ell), both only when m > ell.
__global__ void k_sum_partials(const double* partials, int pstride, int nparts,
                               const int32_t* ranks, int kin, int ell, int what, double* out) {
  const int m = (kin == 0) ? 2 : 2 * ranks[kin];
  if ((what == 0) != (m <= ell)) return;
  const int count = what == 0 ? m * m : (what == 1 ? m * ell : ell * ell);
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

// ---------------------------------------------------------- the small steps
// Q = qr(Y) for a sketched step (m > ell; no-op otherwise): FP64 Householder
// on Y (m x ell, from gy), Q (m x ell) written to gq.
__global__ void __launch_bounds__(kEigThreads) k_sketch_qr(const double* gy, int k, int ell,
                                                           const int32_t* ranks, double* gq) {
  constexpr int NT = kEigThreads, LQ = kSkMaxEll + 1;
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG16 = NT / 16;
  const int m = (k == 1) ? 2 : 2 * ranks[k - 1];
  if (m <= ell) return;  // uniform
  const int el = ell;
  double* Qs = smem;               // m x LQ (Y, then the reflectors, then Q)
  double* bt = Qs + kMaxM * LQ;    // kSkMaxEll
  for (int e = tid; e < m * el; e += NT) {
    const int i = e / el, j = e - i * el;
    Qs[i * LQ + j] = gy[i * ell + j];
  }
  __syncthreads();
  // reflector j overwrites column j (rows j..)
  for (int j = 0; j < el; ++j) {
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
    for (int c = j + 1 + g16; c < el; c += NG16) {
      double d = 0.0;
      for (int i = j + l16; i < m; i += 16) d = fma(Qs[i * LQ + j], Qs[i * LQ + c], d);
      d = sum16(d) * beta;
      for (int i = j + l16; i < m; i += 16) Qs[i * LQ + c] -= d * Qs[i * LQ + j];
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{el-1} [I; 0], formed in place from the last reflector
  for (int j = el - 1; j >= 0; --j) {
    const double beta = bt[j];
    for (int c = j + 1 + g16; c < el; c += NG16) {
      double d = 0.0;
      for (int i = j + l16; i < m; i += 16) d = fma(Qs[i * LQ + j], Qs[i * LQ + c], d);
      d = sum16(d) * beta;
      for (int i = j + l16; i < m; i += 16) Qs[i * LQ + c] -= d * Qs[i * LQ + j];
    }
    __syncthreads();
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
  for (int e = tid; e < m * el; e += NT) {
    const int i = e / el, j = e - i * el;
    gq[e] = Qs[i * LQ + j];
  }
}

// The eigenproblem of step k, the rank rule and core k.  Exact step (m <=
// ell): gy holds the Gram G (m x m), U = its kept eigenvectors.  Sketched
// step: gy holds B B^T (ell x ell), gq the basis Q, U = Q U~_r.  With
// first != 0 (k = 1, always exact) also the norm of the tensor (trace of G)
// and tau^2 into scal.  Writes core k and U (m x r) to umat.
template <typename T>
__global__ void __launch_bounds__(kEigThreads) k_sketch_step(
    const double* gy, const double* gq, int k, int D, double eps, int first, int ell,
    double* scal, int cap_k, T* cores, long long off_k, double* umat, StepOut so) {
  constexpr int NT = kEigThreads, LDA = kEigLds + 1, LQ = kSkMaxEll + 1;
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int rp = (k == 1) ? 1 : so.ranks[k - 1];
  const int m = 2 * rp;
  const bool full = m <= ell;           // uniform
  const int el = full ? m : ell;        // order of the eigenproblem
  double* Qs = smem;                    // m x LQ (sketched steps)
  double* A = Qs + kMaxM * LQ;          // LDA x LDA
  double* V = A + LDA * LDA;            // LDA x LDA
  double* lam = V + LDA * LDA;          // 72
  double* sx = lam + 72;                // kEigScratch
  int* perm = (int*)(sx + kEigScratch); // 72
  int* iscr = perm + 72;                // 8
  if (first && tid == 0) {
    double nrm2 = 0.0;
    for (int i = 0; i < m; ++i) nrm2 += gy[i * m + i];
    scal[0] = nrm2;
    scal[1] = (D > 1) ? eps * eps * nrm2 / (double)(D - 1) : 0.0;
    so.ranks[0] = 1;
  }
  for (int e = tid; e < el * el; e += NT) {
    const int i = e / el, j = e - i * el;
    A[i * LDA + j] = gy[e];
  }
  if (!full) {
    for (int e = tid; e < m * el; e += NT) {
      const int i = e / el, j = e - i * el;
      Qs[i * LQ + j] = gq[e];
    }
  }
  __threadfence();
  __syncthreads();
  // symmetrise (rounding of the partial sums) and solve
  for (int e = tid; e < el * el; e += NT) {
    const int a = e / el, b = e - a * el;
    if (a < b) {
      const double sv = 0.5 * (A[a * LDA + b] + A[b * LDA + a]);
      A[a * LDA + b] = sv;
      A[b * LDA + a] = sv;
    }
  }
  __syncthreads();
  const double tau2 = scal[1];
  const int r = solve_and_truncate<NT>(lds(A), lds(V), el, LDA, lds(sx), lds(iscr), lds(lam),
                                       lds(perm), tau2, cap_k, k, so);
  // U = Q V_r (m x r)
  for (int e = tid; e < m * r; e += NT) {
    const int i = e / r, b = e - i * r;
    double sacc = 0.0;
    if (full) {
      sacc = V[i * LDA + b];
    } else {
      for (int a = 0; a < el; ++a) sacc = fma(Qs[i * LQ + a], V[a * LDA + b], sacc);
    }
    umat[e] = sacc;
    // core k: (a, i, b) <- U[a + rp*i][b]
    const int ii = i / rp, aa = i - ii * rp;
    cores[off_k + (long long)(aa * 2 + ii) * r + b] = (T)sacc;
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
  return sizeof(double) * ((size_t)kMaxM * LQ + 2 * LDA * LDA + 72 + kEigScratch) +
         sizeof(int) * (72 + 8 + 256);
}

static size_t sketch_qr_lds() { return sizeof(double) * ((size_t)kMaxM * (kSkMaxEll + 1) + kSkMaxEll); }

// exact-step Gram partials: kGramParts of kGramPstride doubles (m <= ell <= 64)
constexpr int kGramParts = 512;
constexpr int kGramPstride = kSkMaxEll * kSkMaxEll;

struct SketchPlan {
  double* scal;
  double* partials;
  int pstride;
  double* gy;
  double* gq;
  double* umat;
  void* xbuf[2];
  size_t bytes;
};

static void sketch_plan(int D, int dtype, int ell, void* ws, SketchPlan* p) {
  Arena ar(ws);
  const size_t es = elem_size(dtype);
  p->scal = ar.take<double>(16);
  p->pstride = kMaxM * kMaxM + kMaxM * ell;
  const size_t pe = (size_t)kMaxPartials * p->pstride, ge = (size_t)kGramParts * kGramPstride;
  p->partials = ar.take<double>(pe > ge ? pe : ge);
  p->gy = ar.take<double>((size_t)p->pstride);
  p->gq = ar.take<double>((size_t)kMaxM * kSkMaxEll);
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
    set_lds_limit((const void*)k_sketch_qr, (int)sketch_qr_lds(), &attr_err);
  });
  QTT_HIP_CHECK(attr_err);
  using OT = typename SkOp<BF>::T;
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
  for (int k = 1; k <= D - 1; ++k) {
    const long long n = 1LL << (D - k);
    const int mcap = (k == 1) ? 2 : 2 * cap[k - 1];  // bound on m = 2 r_{k-1}
    const int kin = k - 1;  // ranks index of r_{k-1}; 0 -> m = 2
    const long long nstage = (n + kSkSR - 1) / kSkSR;
    const int blocks = (int)(nstage < kMaxPartials ? nstage : kMaxPartials);
    // 1. exact step (m <= ell): partials of the Gram (no-op on a sketched step),
    // m^2 <= kGramPstride entries each, up to kGramParts of them so that the
    // pass spreads over every compute unit
    const int mg = mcap < ell ? mcap : ell;
    int nparts;
    if (mcap <= 16 && mcap <= ell) {
      // narrow: the Gram in 2048-value stages
      const long long ns2 = (n * mcap + 2047) / 2048;
      nparts = (int)(ns2 < kGramParts ? ns2 : kGramParts);
      ProbeScope _ps(QTT_K_PROJECT, s);
      k_gram_small<T><<<nparts, 256, 0, s>>>(X, n, out.ranks, kin, p.partials, kGramPstride);
    } else {
      nparts = (int)(nstage < kGramParts ? nstage : kGramParts);
      const size_t lds = sizeof(double) * kSkSR * mg;
      ProbeScope _ps(QTT_K_PROJECT, s);
      if (mg <= 16)
        k_gram_sketch<T, 1><<<nparts, 256, lds, s>>>(X, n, out.ranks, kin, ell, p.partials,
                                                     kGramPstride);
      else if (mg <= 32)
        k_gram_sketch<T, 2><<<nparts, 256, lds, s>>>(X, n, out.ranks, kin, ell, p.partials,
                                                     kGramPstride);
      else
        k_gram_sketch<T, 4><<<nparts, 256, lds, s>>>(X, n, out.ranks, kin, ell, p.partials,
                                                     kGramPstride);
    }
    QTT_LAUNCH_CHECK();
    {
      ProbeScope _ps(QTT_K_REDUCE, s);
      k_sum_partials<<<(mg * mg + 255) / 256, 256, 0, s>>>(p.partials, kGramPstride, nparts,
                                                           out.ranks, kin, ell, 0, p.gy);
    }
    QTT_LAUNCH_CHECK();
    // 2. sketched step (m > ell, decided on the device): Y, Q, B B^T
    if (mcap > ell) {
      const int mp = (mcap + 15) & ~15, ep = (ell + 15) & ~15, mk = (mcap + 31) & ~31;
      const size_t lds_y = sizeof(OT) * (size_t)(mp + ep) * kSkLd;
      {
        ProbeScope _ps(QTT_K_SKETCH_GEMM, s);
        k_sketch_y<T, BF><<<blocks, 256, lds_y, s>>>(X, n, out.ranks, kin, ell, k0, k1, k,
                                                     p.partials, p.pstride);
      }
      QTT_LAUNCH_CHECK();
      {
        ProbeScope _ps(QTT_K_REDUCE, s);
        k_sum_partials<<<(mcap * ell + 255) / 256, 256, 0, s>>>(p.partials, p.pstride, blocks,
                                                                out.ranks, kin, ell, 1, p.gy);
      }
      QTT_LAUNCH_CHECK();
      {
        ProbeScope _ps(QTT_K_SKETCH, s);
        k_sketch_qr<<<1, kEigThreads, sketch_qr_lds(), s>>>(p.gy, k, ell, out.ranks, p.gq);
      }
      QTT_LAUNCH_CHECK();
      const size_t lds_b = sizeof(float) * ((size_t)(ep + kSkSR) * (mk + 8) +
                                            (size_t)ep * (kSkSR + 4));
      {
        ProbeScope _ps(QTT_K_SKETCH_GEMM, s);
        k_sketch_gb<T><<<blocks, 256, lds_b, s>>>(X, n, out.ranks, kin, ell, p.gq, p.partials,
                                                  p.pstride);
      }
      QTT_LAUNCH_CHECK();
      {
        ProbeScope _ps(QTT_K_REDUCE, s);
        k_sum_partials<<<(ell * ell + 255) / 256, 256, 0, s>>>(p.partials, p.pstride, blocks,
                                                               out.ranks, kin, ell, 2, p.gy);
      }
      QTT_LAUNCH_CHECK();
    }
    // 3. the small eigenproblem, rank and core k
    {
      ProbeScope _ps(QTT_K_SKETCH, s);
      k_sketch_step<T><<<1, kEigThreads, sketch_step_lds(), s>>>(
          p.gy, p.gq, k, D, eps, k == 1, ell, p.scal, cap[k], cores, out.off[k - 1], p.umat, so);
    }
    QTT_LAUNCH_CHECK();
    // 4. next remainder
    T* Xn = static_cast<T*>(p.xbuf[cur]);
    long long pb = (n * cap[k] + 255) / 256;
    if (pb > 4096) pb = 4096;
    {
      ProbeScope _ps(QTT_K_PROJECT, s);
      k_sketch_project<T><<<(unsigned)pb, 256, 0, s>>>(X, n, out.ranks, kin, k, p.umat, Xn);
    }
    QTT_LAUNCH_CHECK();
    X = Xn;
    cur ^= 1;
  }
  {
    ProbeScope _ps(QTT_K_OTHER, s);
    k_sketch_last<T><<<1, 64, 0, s>>>(X, out.ranks, D, cores, out.off[D - 1], out.ranks);
  }
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

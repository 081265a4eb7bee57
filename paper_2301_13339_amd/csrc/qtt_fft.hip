// QTT-FFT, QTT-iFFT and the QTT-FFT convolution route (Algorithm 2, Step 3;
// Section 4 for the transform, Section 5 for its truncation by max rank,
// tolerance or singular-value drop-off).
//
// The transform is the radix-2 decimation-in-frequency factorisation of the
// DFT taken in TT format.  With the digits of a and b least significant
// first, exp(sigma 2 pi i a b / 2^D) splits into D factors; factor s couples
// output digit b_s with the lowest m = D + 1 - s input digits, so stage s
// sums over a_m: core m becomes the butterfly (slice b = even +- odd), and
// b_s travels along bonds 1..m-1 (which double) into cores 1..m-1, where it
// selects the twiddle exp(sigma i pi 2^(p-m)) on slice a_p = 1.  The output
// is in bit-reversed mode order.
//
// After each stage the doubled bonds are rounded: a left-to-right sweep of
// Householder QRs over cores 1..m-1 (each R absorbed into the next core;
// the doubling and the twiddles are applied while the core is loaded), then
// a right-to-left sweep of SVDs of cores m..2 viewed as r_{p-1} x 2 r_p,
// truncated by the rule of Algorithm 1 with modifications (1) and (3).  Cores
// right of m are right-orthonormal from the previous stage's sweep.  The
// SVDs are one-sided (Hestenes) Jacobi: columns of the core are rotated in
// pairs until orthogonal, so the singular values keep their accuracy (no
// Gram matrix), the rotated columns are U Sigma and the accumulated rotation
// is V.
//
// An image's transform is two-dimensional: the digits of each axis form a
// block transformed by the stages above on its own.  Blocks run right to
// left; a stage doubles only its block's bonds, the QR sweep still starts at
// the first core and the truncation sweep stops at the block, and between
// blocks one LQ makes the first core of the block to the right
// right-orthonormal again (it carried that block's last butterfly).
//
// Every stage of one transform runs in one workgroup (the stages are
// sequential and every matrix is at most 64 x 32 complex); the two forward
// transforms of the convolution run in two workgroups of one launch.  Cores
// live in a workspace slot of fixed stride (bond capacity 32) and stay in
// L2 between stages.  Complex numbers are FP64 pairs (re, im).
#include <math.h>

#include <algorithm>
#include <mutex>

#include "qtt_internal.hpp"
#include "qtt_philox.hpp"
#include "qtt_syev.hpp"

namespace qtt {
namespace fftq {

// complex FP64 value (plain struct: usable through LDS address-space pointers)
struct cplx {
  double x, y;
};
__host__ __device__ __forceinline__ cplx mk(double x, double y) { return cplx{x, y}; }

constexpr int kR = QTT_FFT_MAX_RANK;  // ranks into and out of a transform
constexpr int kB = 2 * kR;            // bond inside a stage (doubled)
constexpr int kSlot = kB * 2 * kB;    // complex entries per core slot
constexpr int kNT = 256;
constexpr int kMaxSweeps = 40;        // Jacobi sweeps (convergence takes 6..10)
constexpr double kJacobiTol = 0x1p-48; // |x^H y| <= tol ||x|| ||y|| ends a pair (32 u)
constexpr int kMaxD = 31;             // modes of a transform (data d <= 30, plus padding)

// ---------------------------------------------------------------- complex
__device__ __forceinline__ cplx cz() { return mk(0.0, 0.0); }
__device__ __forceinline__ cplx cadd(cplx a, cplx b) {
  return mk(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ cplx csub(cplx a, cplx b) {
  return mk(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return mk(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// a * b + c
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx c) {
  return mk(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
// conj(a) * b + c
__device__ __forceinline__ cplx ccfma(cplx a, cplx b, cplx c) {
  return mk(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}
__device__ __forceinline__ cplx cscale(cplx a, double s) {
  return mk(a.x * s, a.y * s);
}
__device__ __forceinline__ cplx cconj(cplx a) { return mk(a.x, -a.y); }
__device__ __forceinline__ double cabs2(cplx a) { return fma(a.x, a.x, a.y * a.y); }

// sum over the 8 lanes l & ~7 .. l | 7 (every lane of the group gets it)
__device__ __forceinline__ double sum8(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  return v;
}
__device__ __forceinline__ cplx csum8(cplx v) {
  return mk(sum8(v.x), sum8(v.y));
}
__device__ __forceinline__ cplx csum16(cplx v) {
  return mk(sum16(v.x), sum16(v.y));
}

__device__ __forceinline__ void barrier_global() {
  __threadfence();
  __syncthreads();
}

// ------------------------------------------------------------ the rule
// Rank kept from n singular values given squared, in non-increasing order:
// smallest r >= 1 with sum_{i>=r} s2_i <= tau2 (Algorithm 1), capped by
// `cap` (modification (1)) and cut at the first sigma_k < delta sigma_{k-1}
// (modification (3)).  *over is set when the rule without the cap wanted
// more than the cap.
__device__ inline int rule_rank(lds_ptr<const double> s2, int n, double tau2, int cap,
                                double delta, int* over) {
  // tail(r) = sum_{i >= r} s2_i grows as r falls; scan from the small end
  int r = n;
  double tail = 0.0;
  for (int c = n - 1; c >= 1; --c) {
    tail += s2[c];
    if (tail <= tau2)
      r = c;
    else
      break;
  }
  if (delta > 0.0) {
    for (int k = 1; k < n; ++k)
      if (sqrt(s2[k]) < delta * sqrt(s2[k - 1])) {
        r = min(r, k);
        break;
      }
  }
  *over = r > cap;
  r = min(r, cap);
  return max(r, 1);
}

// ------------------------------------------------------- Householder QR
// QR of the M x N complex matrix (M <= 64, N <= 32) held by column: thread t
// owns column t >> 3, rows 8 (t & 7) + e in a[e].  Reflector j is
// H_j = I - (2 / v^H v) v v^H with v = x - alpha e_j, alpha = -phase(x_j)
// ||x|| (x the column below row j), stored in sV[j][*].  On return a[] holds
// column c < K of Q = H_0 ... H_{K-1} [I_K; 0], K = min(M, N), and sR (row
// stride kB) the K x N factor R (zero below the diagonal).  One barrier per
// reflector; the caller synchronises before reading sR.
__device__ __forceinline__ void house_qr(cplx a[8], int M, int N, cplx* sV, lds_ptr<double> sVV,
                         cplx* sR) {
  const int t = threadIdx.x, c = t >> 3, q = t & 7;
  const int K = min(M, N);
  for (int j = 0; j < K; ++j) {
    if (c == j) {
      double n2 = 0.0;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int row = 8 * q + e;
        if (row >= j && row < M) n2 += cabs2(a[e]);
      }
      n2 = sum8(n2);
      // x_j from its owner lane through LDS (the group is one wave, whose
      // LDS accesses complete in order)
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (8 * q + e == j) sV[j * 64 + j] = a[e];
      __builtin_amdgcn_wave_barrier();
      const cplx x0 = sV[j * 64 + j];
      __builtin_amdgcn_wave_barrier();
      const double sig = sqrt(n2);
      const double xa = sqrt(cabs2(x0));
      cplx alpha = cz();
      double vv = 0.0;
      if (sig > 0.0) {
        const cplx ph = xa > 0.0 ? cscale(x0, 1.0 / xa) : mk(1.0, 0.0);
        alpha = cscale(ph, -sig);
        vv = 2.0 * sig * (sig + xa);
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int row = 8 * q + e;
        cplx v = cz();
        if (row >= j && row < M) v = (row == j) ? csub(a[e], alpha) : a[e];
        sV[j * 64 + row] = v;
      }
      if (q == 0) {
        sVV[j] = vv;
        sR[j * kB + j] = alpha;
      }
      for (int i = j + 1 + q; i < K; i += 8) sR[i * kB + j] = cz();
    }
    __syncthreads();
    if (c > j && c < N) {
      const double vv = sVV[j];
      if (vv > 0.0) {
        cplx w = cz();
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int row = 8 * q + e;
          if (row >= j && row < M) w = ccfma(sV[j * 64 + row], a[e], w);
        }
        w = csum8(w);
        const double f = 2.0 / vv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int row = 8 * q + e;
          if (row >= j && row < M) a[e] = csub(a[e], cscale(cmul(sV[j * 64 + row], w), f));
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (8 * q + e == j) sR[j * kB + c] = a[e];
    }
  }
  // Q = H_0 ... H_{K-1} [I; 0], applied from the last reflector; columns
  // below j are untouched by H_j (they vanish in rows >= j)
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int row = 8 * q + e;
    a[e] = (row == c && c < K) ? mk(1.0, 0.0) : cz();
  }
  for (int j = K - 1; j >= 0; --j) {
    if (c >= j && c < K) {
      const double vv = sVV[j];
      if (vv > 0.0) {
        cplx w = cz();
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int row = 8 * q + e;
          if (row >= j && row < M) w = ccfma(sV[j * 64 + row], a[e], w);
        }
        w = csum8(w);
        const double f = 2.0 / vv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int row = 8 * q + e;
          if (row >= j && row < M) a[e] = csub(a[e], cscale(cmul(sV[j * 64 + row], w), f));
        }
      }
    }
  }
}

// ------------------------------------------------------ one-sided Jacobi
// C (M x N, M <= 32, N <= 32 and even) by column in sC (column c at
// sC[c * kB]): on return sC holds W = C J with mutually orthogonal columns
// (their norms are the singular values) and sJ (column-major, stride kB) the
// unitary J.  The N/2 disjoint pairs of a round (circle schedule) are
// rotated at once, 16 lanes per pair; a sweep is N-1 rounds.  A pair (x, y)
// with g = x^H y = |g| e is rotated by x' = c x - s conj(e) y,
// y' = s e x + c y, with t = s / c the smaller root of
// t^2 + 2 zeta t - 1 = 0, zeta = (|y|^2 - |x|^2) / (2 |g|), which makes
// x'^H y' = 0.
__device__ __forceinline__ void jacobi(cplx* sC, cplx* sJ, int M, int N, lds_ptr<int> sFlag,
                                       lds_ptr<double> s2, lds_ptr<double> scal) {
  const int t = threadIdx.x, g = t >> 4, h = t & 15;
  for (int i = t; i < kB * kB; i += kNT) {
    const int row = i % kB, col = i / kB;
    sJ[i] = (row == col && col < N) ? mk(1.0, 0.0) : cz();
  }
  if (t < 3) sFlag[t] = 0;
  // ||C||_F^2 (invariant under the rotations): a pair with a column below
  // 2^-52 ||C||_F is left alone, since rotating rounding-level columns
  // against each other never meets the relative test
  for (int c = g; c < N; c += 16) {
    double v = 0.0;
    if (h < M) v += cabs2(sC[c * kB + h]);
    if (h + 16 < M) v += cabs2(sC[c * kB + h + 16]);
    v = sum16(v);
    if (h == 0) s2[c] = v;
  }
  __syncthreads();
  if (t == 0) {
    double f2 = 0.0;
    for (int c = 0; c < N; ++c) f2 += s2[c];
    scal[1] = f2 * 0x1p-104;
  }
  __syncthreads();
  const double tiny2 = scal[1];
  const int P = N / 2;
  const double tol2 = kJacobiTol * kJacobiTol;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    if (t == 0) sFlag[(sweep + 1) % 3] = 0;
    for (int rd = 0; rd < N - 1; ++rd) {
      if (g < P) {
        int ia = g - 1 + rd, ib = N - 2 - g + rd;  // both below 2 (N - 1)
        if (ia >= N - 1) ia -= N - 1;
        if (ib >= N - 1) ib -= N - 1;
        const int a = (g == 0) ? 0 : 1 + ia;
        const int b = 1 + ib;
        cplx x0 = cz(), x1 = cz(), y0 = cz(), y1 = cz();
        if (h < M) {
          x0 = sC[a * kB + h];
          y0 = sC[b * kB + h];
        }
        if (h + 16 < M) {
          x1 = sC[a * kB + h + 16];
          y1 = sC[b * kB + h + 16];
        }
        const double al = sum16(cabs2(x0) + cabs2(x1));
        const double be = sum16(cabs2(y0) + cabs2(y1));
        const cplx gm = csum16(ccfma(x0, y0, ccfma(x1, y1, cz())));
        const double g2 = cabs2(gm);
        if (g2 > 0.0 && g2 > tol2 * al * be && al > tiny2 && be > tiny2) {
          // Newton-refined hardware estimates instead of divisions and
          // square roots: the rotation stays exactly unitary to rounding
          // (cs and sn come from one t), only t's last bits differ
          const double ig = rsq_acc(g2);
          const cplx e = cscale(gm, ig);
          const double zeta = 0.5 * (be - al) * ig;
          const double az = fabs(zeta);
          double tt;
          if (az < 1e100) {
            const double z2 = fma(zeta, zeta, 1.0);
            tt = rcp_acc(az + z2 * rsq_acc(z2));
          } else {
            tt = 0.5 / az;
          }
          if (zeta < 0.0) tt = -tt;
          const double cs = rsq_acc(fma(tt, tt, 1.0));
          const double sn = cs * tt;
          const cplx se = cscale(e, sn), sec = cconj(se);
          if (h < M) {
            sC[a * kB + h] = csub(cscale(x0, cs), cmul(sec, y0));
            sC[b * kB + h] = cfma(se, x0, cscale(y0, cs));
          }
          if (h + 16 < M) {
            sC[a * kB + h + 16] = csub(cscale(x1, cs), cmul(sec, y1));
            sC[b * kB + h + 16] = cfma(se, x1, cscale(y1, cs));
          }
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            const int row = h + 16 * half;
            if (row < N) {
              const cplx jx = sJ[a * kB + row], jy = sJ[b * kB + row];
              sJ[a * kB + row] = csub(cscale(jx, cs), cmul(sec, jy));
              sJ[b * kB + row] = cfma(se, jx, cscale(jy, cs));
            }
          }
          if (h == 0) sFlag[sweep % 3] = 1;
        }
      }
      __syncthreads();
    }
    if (sFlag[sweep % 3] == 0) break;
  }
}

// squared column norms of W (N columns, M rows) into s2; then the order of
// the columns by non-increasing norm into perm and the sorted squares into
// s2s (first n = min(M, N)).  Two barriers.
__device__ __forceinline__ void sort_columns(const cplx* sC, int M, int N, lds_ptr<double> s2,
                             lds_ptr<double> s2s, lds_ptr<int> perm) {
  const int t = threadIdx.x, g = t >> 4, h = t & 15;
  for (int c = g; c < N; c += 16) {
    double v = 0.0;
    if (h < M) v += cabs2(sC[c * kB + h]);
    if (h + 16 < M) v += cabs2(sC[c * kB + h + 16]);
    v = sum16(v);
    if (h == 0) s2[c] = v;
  }
  __syncthreads();
  if (t < N) {
    const double mine = s2[t];
    int rank = 0;
    for (int c = 0; c < N; ++c) {
      const double o = s2[c];
      rank += (o > mine) || (o == mine && c < t);
    }
    perm[rank] = t;
    s2s[rank] = mine;
  }
  __syncthreads();
}

// ---------------------------------------------------------------- tasks
struct Task {
  cplx* cores;    // engine layout: core p (0-based) at p * kSlot
  int32_t* ranks;    // r_0..r_D
  int32_t* status;   // may be null
  int D;
  int sign;          // -1 forward, +1 inverse exponent
  int cap;           // rank cap (1..kR)
  int lib_cap;       // 1: the cap is the library's, flag when the rule wanted more
  double eps;        // tolerance of each rounding (0 = off)
  double delta;      // drop-off threshold (0 = off)
  int nblk;          // axes: blocks of consecutive cores, each transformed on its own
  int lo[2], hi[2];  // 0-based first core and end of each block
};
struct Tasks {
  Task t[2];
};

struct Smem {
  cplx V[kB * 64];      // reflectors
  cplx R[kB * kB];      // QR factor R (row stride kB)
  cplx C[2][kB * kB];   // Jacobi matrix, column-major, two buffers
  cplx J[kB * kB];      // Jacobi rotations, column-major
  double VV[kB];
  double s2[kB];
  double s2s[kB];
  double scal[4];
  int perm[kB];
  int rk[kMaxD + 1];       // current ranks
  int r0[kMaxD + 1];       // ranks before the stage
  int flag[4];
  int over;
};

// Right-to-left truncation sweep from core m (whose right unfolding, M x
// 2 rr, is in S.C[0]) down to core lo + 2; cores 1..m-1 are left-orthonormal
// and cores right of m right-orthonormal.  Truncates bonds m-1..lo+1 with
// tau^2 = eps^2 ||centre||^2 / (D-1) and writes cores m..lo+1.
__device__ __forceinline__ void svd_sweep(const Task& T, int m, int M, int rr, int lo, Smem& S) {
  const int t = threadIdx.x;
  const int D = T.D;
  cplx* const tc = T.cores;
  auto slot = [=](int p) { return tc + (size_t)(p - 1) * kSlot; };
  int cur = 0;
  for (int p = m; p >= lo + 2; --p) {
    const int N = 2 * rr;
    jacobi(S.C[cur], S.J, M, N, lds(S.flag), lds(S.s2), lds(S.scal));
    sort_columns(S.C[cur], M, N, lds(S.s2), lds(S.s2s), lds(S.perm));
    if (t == 0) {
      if (p == m) {
        double nrm2 = 0.0;
        for (int i = 0; i < N; ++i) nrm2 += S.s2[i];
        S.scal[0] = D > 1 ? T.eps * T.eps * nrm2 / (double)(D - 1) : 0.0;
      }
      int over = 0;
      const int r = rule_rank(lds((const double*)S.s2s), min(M, N), S.scal[0], T.cap, T.delta,
                              &over);
      if (over && T.lib_cap && T.status) atomicOr(T.status, QTT_STATUS_RANKCAP);
      S.rk[p - 1] = r;
    }
    __syncthreads();
    const int r = S.rk[p - 1];
    // core p = rows perm[0..r) of J^H, shape (r, 2, rr)
    cplx* Gw = slot(p);
    for (int idx = t; idx < r * N; idx += kNT) {
      const int j = idx / N, col = idx - j * N;  // col = i * rr + beta
      Gw[j * N + col] = cconj(S.J[S.perm[j] * kB + col]);
    }
    // new centre p-1: Q_{p-1} (Ml, 2, M) times W[:, perm[0..r)]
    const int Ml = S.rk[p - 2];  // r_0 = 1
    const cplx* Q = slot(p - 1);
    const int nxt = cur ^ 1;
    for (int idx = t; idx < Ml * 2 * r; idx += kNT) {
      const int a = idx % Ml, col = idx / Ml;  // col = i * r + j
      const int i = col / r, j = col - i * r;
      cplx v = cz();
      const int pc = S.perm[j];
      for (int cc = 0; cc < M; ++cc) v = cfma(Q[(a * 2 + i) * M + cc], S.C[cur][pc * kB + cc], v);
      S.C[nxt][col * kB + a] = v;
    }
    barrier_global();
    cur = nxt;
    rr = r;
    M = Ml;
  }
  // the last centre is core lo + 1, (r_lo, 2, rr)
  cplx* G1 = slot(lo + 1);
  for (int idx = t; idx < M * 2 * rr; idx += kNT) {
    const int a = idx % M, col = idx / M;
    G1[a * 2 * rr + col] = S.C[cur][col * kB + a];
  }
  barrier_global();
}

// the stage whose summed digit sits at core m (1-based, m >= lo + 2, the
// block starting at 0-based core lo) and the rounding of its doubled bonds
__device__ __forceinline__ void stage_and_round(const Task& T, int m, int lo, Smem& S) {
  const int t = threadIdx.x, c = t >> 3, q = t & 7;
  const int D = T.D;
  cplx* const tc = T.cores;
  auto slot = [=](int p) { return tc + (size_t)(p - 1) * kSlot; };  // 1-based core
  if (t <= D) S.r0[t] = S.rk[t];
  __syncthreads();
  // ---- left-to-right QR sweep over cores 1..m-1; the bonds of cores
  // lo+1..m-1 double (the first of them keeps its left bond)
  int k = 1;  // rows (left bond) of the current R
  for (int p = 1; p < m; ++p) {
    const int rl = S.r0[p - 1], rr = S.r0[p];
    const bool dl = p > lo + 1, dr = p > lo;
    const int M = 2 * k, N = dr ? 2 * rr : rr;
    cplx wtw;  // twiddle on slice 1 of branch k' = 1
    {
      double sn, cs;
      sincospi(ldexp(1.0, p - m), &sn, &cs);
      wtw = mk(cs, T.sign * sn);
    }
    const cplx* G = slot(p);
    cplx a[8];
    const int kp = dr ? c / max(rr, 1) : 0, beta = c - kp * rr;
    const int roff = dl ? kp * rl : 0;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int row = 8 * q + e;
      cplx v = cz();
      if (row < M && c < N) {
        const int cp = row >> 1, i = row & 1;
        if (p == 1) {
          v = G[i * rr + beta];
        } else {
          for (int al = 0; al < rl; ++al)
            v = cfma(S.R[cp * kB + roff + al], G[(al * 2 + i) * rr + beta], v);
        }
        if (kp == 1 && i == 1) v = cmul(v, wtw);
      }
      a[e] = v;
    }
    __syncthreads();  // everyone has read R
    house_qr(a, M, N, S.V, lds(S.VV), S.R);
    const int kn = min(M, N);
    cplx* Gw = slot(p);
    if (c < kn) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int row = 8 * q + e;
        if (row < M) Gw[row * kn + c] = a[e];  // (cp, i, c) at (cp*2+i)*kn + c
      }
    }
    if (t == 0) S.rk[p] = kn;
    k = kn;
    barrier_global();
  }
  // ---- the centre: R times the butterfly of core m
  {
    const int rl = S.r0[m - 1], rr = S.r0[m];
    const cplx* G = slot(m);
    const int N = 2 * rr;
    for (int idx = t; idx < k * N; idx += kNT) {
      const int cp = idx % k, col = idx / k;
      const int b = col / rr, beta = col - b * rr;
      cplx v = cz();
      for (int al = 0; al < rl; ++al) {
        const cplx h0 = G[(al * 2) * rr + beta], h1 = G[(al * 2 + 1) * rr + beta];
        const cplx hb = b ? csub(h0, h1) : cadd(h0, h1);
        v = cfma(S.R[cp * kB + b * rl + al], hb, v);
      }
      S.C[0][col * kB + cp] = v;
    }
  }
  __syncthreads();
  svd_sweep(T, m, k, S.r0[m], lo, S);
}

// Core p0 + 1 (1-based) made right-orthonormal: Householder QR of its
// conjugate-transposed right unfolding C^H = Q R (C = R^H Q^H), the core
// becomes Q^H and R^H is absorbed into core p0.
__device__ __forceinline__ void right_orth(const Task& T, int p0, Smem& S) {
  const int t = threadIdx.x, c = t >> 3, q = t & 7;
  cplx* const tc = T.cores;
  cplx* Gc = tc + (size_t)p0 * kSlot;           // the core made right-orthonormal
  cplx* Gl = tc + (size_t)(p0 - 1) * kSlot;     // its left neighbour
  const int rl = S.rk[p0], rr = S.rk[p0 + 1], rll = S.rk[p0 - 1];
  const int M = 2 * rr, N = rl;
  cplx a[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int row = 8 * q + e;  // row = i * rr + b of C^H, column c = a of C
    cplx v = cz();
    if (row < M && c < N) {
      const int i = row / rr, b = row - i * rr;
      v = cconj(Gc[(c * 2 + i) * rr + b]);
    }
    a[e] = v;
  }
  __syncthreads();
  house_qr(a, M, N, S.V, lds(S.VV), S.R);
  const int K = min(M, N);
  __syncthreads();
  if (c < K) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int row = 8 * q + e;
      if (row < M) {
        const int i = row / rr, b = row - i * rr;
        Gc[(c * 2 + i) * rr + b] = cconj(a[e]);
      }
    }
  }
  // left neighbour times R^H, through LDS (read all, then write)
  for (int idx = t; idx < rll * 2 * K; idx += kNT) {
    const int j = idx % K, ai = idx / K;  // ai = alpha * 2 + i
    cplx v = cz();
    for (int x = 0; x < N; ++x) v = ccfma(S.R[j * kB + x], Gl[ai * rl + x], v);
    S.C[0][idx] = v;
  }
  __syncthreads();
  for (int idx = t; idx < rll * 2 * K; idx += kNT) Gl[idx] = S.C[0][idx];
  if (t == 0) S.rk[p0] = K;
  barrier_global();
}

__global__ __launch_bounds__(kNT) void k_qfft(Tasks tasks) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Smem& S = *reinterpret_cast<Smem*>(smem_raw);
  const Task T = blockIdx.x == 0 ? tasks.t[0] : tasks.t[1];
  const int t = threadIdx.x, D = T.D;
  if (t <= D) S.rk[t] = T.ranks[t];
  __syncthreads();
  for (int bi = T.nblk - 1; bi >= 0; --bi) {
    const int lo = bi == 0 ? T.lo[0] : T.lo[1], hi = bi == 0 ? T.hi[0] : T.hi[1];
    if (bi < T.nblk - 1) right_orth(T, T.lo[1], S);
    for (int m = hi; m >= lo + 1; --m) {
      if (m >= lo + 2) {
        stage_and_round(T, m, lo, S);
      } else {
        // the block's last stage: butterfly of core lo + 1, no bond doubles
        const int rl = S.rk[lo], rr = S.rk[lo + 1];
        cplx* G = T.cores + (size_t)lo * kSlot;
        cplx ev = cz(), od = cz();
        const int al = t / max(rr, 1), be = t - al * rr;
        if (t < rl * rr) {
          const cplx g0 = G[(al * 2) * rr + be], g1 = G[(al * 2 + 1) * rr + be];
          ev = cadd(g0, g1);
          od = csub(g0, g1);
        }
        __syncthreads();
        if (t < rl * rr) {
          G[(al * 2) * rr + be] = ev;
          G[(al * 2 + 1) * rr + be] = od;
        }
        barrier_global();
      }
    }
  }
  if (t <= D) T.ranks[t] = S.rk[t];
}

// ------------------------------------------------- Hadamard product rounding
// Randomised rounding of the entrywise product H = A . B of two spectra
// ("randomize then orthogonalize", Al Daas et al., SIAM J. Sci. Comput.
// 2023): with a Gaussian TT Omega of ranks ell (Philox entries; core p,
// 1-based, has entry (t, i, u) from row 2t + i, column u, step p), the right
// sketches W_{p-1} = sum_i H_p[:, i, :] W_p Omega_p[:, i, :]^T are formed
// right to left (W_D = 1) without forming H, using H_p = A_p (x) B_p slice
// by slice; then left to right M = Z H_p, Y = M W_{p+1}, Y = Q R,
// core p = Q, Z = Q^H M; the last core is Z H_D.  Cores 1..D-1 are then
// left-orthonormal and the truncation sweep of the transforms follows.
constexpr int kL = QTT_FFT_MAX_ELL;   // largest sketch width
constexpr int kHad = kR * kR;         // largest product rank

struct HadArgs {
  const cplx* A;
  const int32_t* ra;
  const cplx* Bm;
  const int32_t* rb;
  Task out;           // result tensor (engine layout) and truncation rule
  cplx* W;         // D sketches, each kHad x kL (row stride kL)
  cplx* Mb;        // 2 kL x kHad (also the 2 x kHad x kL stage of the sketches)
  cplx* T1;        // kL x kR x 2 x kR
  cplx* Zb;        // kL x kHad
  int ell;
  uint32_t k0, k1;    // seed words
};

struct HadSmem {
  Smem s;
  double om[2 * kL * kL];
};

__global__ __launch_bounds__(kNT) void k_had_round(HadArgs H) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  HadSmem& SS = *reinterpret_cast<HadSmem*>(smem_raw);
  Smem& S = SS.s;
  const int t = threadIdx.x, c = t >> 3, q = t & 7;
  const Task T = H.out;
  const int D = T.D, ell = H.ell;
  const cplx* const hA = H.A;
  const cplx* const hB = H.Bm;
  cplx* const hW = H.W;
  cplx* const oc = T.cores;
  auto A = [=](int p) { return hA + (size_t)p * kSlot; };   // 0-based core
  auto Bc = [=](int p) { return hB + (size_t)p * kSlot; };
  auto Wp = [=](int p) { return hW + (size_t)p * kHad * kL; };
  auto out = [=](int p) { return oc + (size_t)p * kSlot; };
  // ---- right-to-left sketches
  if (t == 0) Wp(D)[0] = mk(1.0, 0.0);
  barrier_global();
  for (int p = D - 1; p >= 1; --p) {
    const int la = ell, lb = (p == D - 1) ? 1 : ell;
    const int rA0 = H.ra[p], rA1 = H.ra[p + 1], rB0 = H.rb[p], rB1 = H.rb[p + 1];
    const int Y1 = rA1 * rB1;
    for (int idx = t; idx < 2 * la * lb; idx += kNT) {
      const int row = idx / lb, u = idx - row * lb;  // row = 2 t + i
      SS.om[idx] = omega_entry(row, u, p + 1, H.k0, H.k1);
    }
    __syncthreads();
    // V_i[y, tt] = sum_u W_{p+1}[y, u] Omega[tt, i, u]
    const cplx* Wn = Wp(p + 1);
    for (int idx = t; idx < 2 * Y1 * la; idx += kNT) {
      const int tt = idx % la, rest = idx / la, y = rest % Y1, i = rest / Y1;
      cplx v = cz();
      for (int u = 0; u < lb; ++u) {
        const double o = SS.om[(tt * 2 + i) * lb + u];
        const cplx w = Wn[y * kL + u];
        v.x = fma(w.x, o, v.x);
        v.y = fma(w.y, o, v.y);
      }
      H.Mb[idx] = v;  // ((i * Y1 + y) * la + tt)
    }
    barrier_global();
    // X_i[(a, b'), tt] = sum_b A_p[a, i, b] V_i[(b, b'), tt]
    const cplx* Ap = A(p);
    for (int idx = t; idx < 2 * rA0 * rB1 * la; idx += kNT) {
      const int tt = idx % la, r1 = idx / la, bp = r1 % rB1, r2 = r1 / rB1, a = r2 % rA0,
                i = r2 / rA0;
      cplx v = cz();
      for (int b = 0; b < rA1; ++b)
        v = cfma(Ap[(a * 2 + i) * rA1 + b], H.Mb[((i * Y1) + b * rB1 + bp) * la + tt], v);
      H.T1[idx] = v;  // (((i * rA0 + a) * rB1 + b') * la + tt)
    }
    barrier_global();
    // W_p[(a, a'), tt] = sum_i sum_b' B_p[a', i, b'] X_i[(a, b'), tt]
    const cplx* Bp = Bc(p);
    cplx* Wc = Wp(p);
    for (int idx = t; idx < rA0 * rB0 * la; idx += kNT) {
      const int tt = idx % la, x = idx / la, a = x / rB0, ap = x - a * rB0;
      cplx v = cz();
      for (int i = 0; i < 2; ++i)
        for (int bp = 0; bp < rB1; ++bp)
          v = cfma(Bp[(ap * 2 + i) * rB1 + bp], H.T1[(((i * rA0 + a) * rB1) + bp) * la + tt], v);
      Wc[x * kL + tt] = v;
    }
    barrier_global();
  }
  // ---- left to right: orthonormal cores from the sketched unfoldings
  if (t == 0) H.Zb[0] = mk(1.0, 0.0);
  if (t == 0) S.rk[0] = 1;
  barrier_global();
  int k = 1;
  for (int p = 0; p < D - 1; ++p) {
    const int rA0 = H.ra[p], rA1 = H.ra[p + 1], rB0 = H.rb[p], rB1 = H.rb[p + 1];
    const int X1 = rA1 * rB1;
    const cplx* Ap = A(p);
    const cplx* Bp = Bc(p);
    // T1[c, a', i, b] = sum_a Z[c, (a, a')] A_p[a, i, b]
    for (int idx = t; idx < k * rB0 * 2 * rA1; idx += kNT) {
      const int b = idx % rA1, r1 = idx / rA1, i = r1 & 1, r2 = r1 >> 1, ap = r2 % rB0,
                cc = r2 / rB0;
      cplx v = cz();
      for (int a = 0; a < rA0; ++a)
        v = cfma(H.Zb[cc * kHad + a * rB0 + ap], Ap[(a * 2 + i) * rA1 + b], v);
      H.T1[idx] = v;  // (((cc * rB0 + a') * 2 + i) * rA1 + b)
    }
    barrier_global();
    // M[(c, i), (b, b')] = sum_a' T1[c, a', i, b] B_p[a', i, b']
    for (int idx = t; idx < 2 * k * X1; idx += kNT) {
      const int y = idx % X1, row = idx / X1, i = row & 1, cc = row >> 1;
      const int b = y / rB1, bp = y - b * rB1;
      cplx v = cz();
      for (int ap = 0; ap < rB0; ++ap)
        v = cfma(H.T1[((cc * rB0 + ap) * 2 + i) * rA1 + b], Bp[(ap * 2 + i) * rB1 + bp], v);
      H.Mb[row * kHad + y] = v;
    }
    barrier_global();
    // Y = M W_{p+1} (2k x ell) into the QR layout
    const cplx* Wn = Wp(p + 1);
    const int M = 2 * k, N = ell;
    cplx a[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int row = 8 * q + e;
      cplx v = cz();
      if (row < M && c < N)
        for (int y = 0; y < X1; ++y) v = cfma(H.Mb[row * kHad + y], Wn[y * kL + c], v);
      a[e] = v;
    }
    __syncthreads();
    house_qr(a, M, N, S.V, lds(S.VV), S.R);
    const int kn = min(M, N);
    cplx* G = out(p);
    if (c < kn) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int row = 8 * q + e;
        if (row < M) G[row * kn + c] = a[e];
      }
    }
    if (t == 0) S.rk[p + 1] = kn;
    barrier_global();
    // Z = Q^H M (kn x X1)
    for (int idx = t; idx < kn * X1; idx += kNT) {
      const int y = idx % X1, cc = idx / X1;
      cplx v = cz();
      for (int row = 0; row < M; ++row) v = ccfma(G[row * kn + cc], H.Mb[row * kHad + y], v);
      H.Zb[cc * kHad + y] = v;
    }
    barrier_global();
    k = kn;
  }
  // last core Z H_D, shape (k, 2, 1), straight into the centre buffer
  {
    const int p = D - 1;
    const int rA0 = H.ra[p], rB0 = H.rb[p];
    const cplx* Ap = A(p);
    const cplx* Bp = Bc(p);
    for (int idx = t; idx < 2 * k; idx += kNT) {
      const int cc = idx % k, i = idx / k;
      cplx v = cz();
      for (int a = 0; a < rA0; ++a)
        for (int ap = 0; ap < rB0; ++ap)
          v = cfma(H.Zb[cc * kHad + a * rB0 + ap], cmul(Ap[a * 2 + i], Bp[ap * 2 + i]), v);
      S.C[0][i * kB + cc] = v;
    }
    if (t == 0) S.rk[D] = 1;
  }
  __syncthreads();
  svd_sweep(T, D, k, 1, 0, S);
  if (t <= D) T.ranks[t] = S.rk[t];
}

// ----------------------------------------------------- layout conversions
// Cores of a source tensor into the engine layout (complex, slot stride
// kSlot) from engine core `core0` on: optionally with the mode order
// reversed, a zero-padding mode inserted before source core `pad_mid`
// (identity core, slice 1 zero) and one appended at the end (slice 1 zero),
// the source's top core's slices swapped (rotation by half the length) and
// the first core scaled.
struct LoadArgs {
  const void* src;
  int kind;                     // 0 f32, 1 f64, 2 complex FP64 pairs
  const int32_t* src_ranks;
  long long off[kMaxD + 1];     // element offsets of the source cores
  int d_src;
  cplx* dst;
  int32_t* dst_ranks;
  int core0;                    // first engine core written
  int ncores;                   // engine cores written (d_src + the padding cores)
  int reverse, pad_mid, pad_end, rotate;
  double scale;
  int32_t* status;              // QTT_STATUS_FFT_RANK when a source rank is too large
};

__device__ __forceinline__ cplx load_elem(const void* src, int kind, long long i) {
  if (kind == 0) return mk((double)static_cast<const float*>(src)[i], 0.0);
  if (kind == 1) return mk(static_cast<const double*>(src)[i], 0.0);
  return static_cast<const cplx*>(src)[i];
}

// rank of bond j (0..ncores) of the written cores
__device__ __forceinline__ int load_rank(const LoadArgs& L, int j) {
  if (L.pad_end && j == L.ncores) return 1;
  if (L.pad_mid >= 0 && j == L.pad_mid + 1) return L.src_ranks[L.pad_mid];
  const int sj = j - ((L.pad_mid >= 0 && j > L.pad_mid) ? 1 : 0);
  return L.reverse ? L.src_ranks[L.d_src - sj] : L.src_ranks[sj];
}

__global__ void k_fft_load(LoadArgs L) {
  // a rank above the engine's limit: the tensor is replaced by zero (ranks
  // 1) and the condition reported, so that every later kernel stays inside
  // its slots
  bool bad = false;
  for (int j = 0; j <= L.d_src; ++j) bad |= L.src_ranks[j] > kR || L.src_ranks[j] < 1;
  const long long g0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  cplx* const dst = L.dst + (size_t)L.core0 * kSlot;
  if (bad) {
    if (g0 < L.ncores) {
      dst[g0 * kSlot] = mk(0.0, 0.0);
      dst[g0 * kSlot + 1] = mk(0.0, 0.0);
    }
    if (g0 <= L.ncores) L.dst_ranks[L.core0 + g0] = 1;
    if (g0 == 0 && L.status) atomicOr(L.status, QTT_STATUS_FFT_RANK);
    return;
  }
  const long long total = (long long)L.ncores * kSlot;
  for (long long g = g0; g < total; g += (long long)gridDim.x * blockDim.x) {
    const int p = (int)(g / kSlot), e = (int)(g - (long long)p * kSlot);
    if (L.pad_end && p == L.ncores - 1) {
      if (e < 2) dst[g] = mk(e == 0 ? 1.0 : 0.0, 0.0);
      continue;
    }
    if (p == L.pad_mid) {
      const int r = L.src_ranks[L.pad_mid];
      if (e < r * 2 * r) {
        const int a = e / (2 * r), i = (e / r) & 1, b = e % r;
        dst[g] = mk((i == 0 && a == b) ? 1.0 : 0.0, 0.0);
      }
      continue;
    }
    const int q = p - ((L.pad_mid >= 0 && p > L.pad_mid) ? 1 : 0);  // source core
    const int sp = L.reverse ? L.d_src - 1 - q : q;
    const int s0 = L.src_ranks[sp], s1 = L.src_ranks[sp + 1];
    const int d0 = L.reverse ? s1 : s0, d1 = L.reverse ? s0 : s1;
    if (e >= d0 * 2 * d1) continue;
    const int a = e / (2 * d1), i = (e / d1) & 1, b = e % d1;
    const int sa = L.reverse ? b : a, sb = L.reverse ? a : b;
    const int si = (L.rotate && sp == L.d_src - 1) ? 1 - i : i;
    cplx v = load_elem(L.src, L.kind, L.off[sp] + (long long)(sa * 2 + si) * s1 + sb);
    if (p == 0) v = cscale(v, L.scale);
    dst[g] = v;
  }
  if (g0 <= L.ncores) L.dst_ranks[L.core0 + g0] = load_rank(L, (int)g0);
}

// An engine tensor (D modes) into a caller's tensor: optionally the mode
// order reversed and the first core scaled (the inverse transform's output),
// the slices with padding digit 0 taken (mode `mid` and, with `lower`, the
// last mode: the lower half of the circular convolution on each axis), and
// the real part as a real TT (interior cores [[Re, -Im], [Im, Re]], bond
// index s * r + alpha, first core its first block row, last core its first
// block column).
struct StoreArgs {
  const cplx* src;
  const int32_t* src_ranks;
  int D;
  int reverse, lower, realify;
  int mid;                      // logical core of an inner padding digit, or -1
  double scale;
  void* dst;
  int kind;                     // 0 f32, 1 f64, 2 complex
  int32_t* dst_ranks;
  long long off[kMaxD + 1];
  int cap[kMaxD + 1];
};

// rank j of the logical source (reversed as asked)
__device__ __forceinline__ int lrank(const StoreArgs& S, int j) {
  return S.reverse ? S.src_ranks[S.D - j] : S.src_ranks[j];
}
// entry (a, i, b) of logical core p (reversed and scaled as asked)
__device__ __forceinline__ cplx lentry(const StoreArgs& S, int p, int a, int i, int b) {
  cplx v;
  if (S.reverse) {
    const int sp = S.D - 1 - p, r1 = S.src_ranks[sp + 1];
    v = S.src[(size_t)sp * kSlot + (b * 2 + i) * r1 + a];
  } else {
    v = S.src[(size_t)p * kSlot + (a * 2 + i) * lrank(S, p + 1) + b];
  }
  return p == 0 ? cscale(v, S.scale) : v;
}
// logical core of output core p, and the logical rank of output bond j
__device__ __forceinline__ int lcore(const StoreArgs& S, int p) {
  return p + ((S.mid >= 0 && p >= S.mid) ? 1 : 0);
}
__device__ __forceinline__ int obond(const StoreArgs& S, int j) {
  return lrank(S, j + ((S.mid >= 0 && j >= S.mid) ? 1 : 0));
}
// entry of the logical core lp with the padding digits contracted at 0
__device__ __forceinline__ cplx centry(const StoreArgs& S, int lp, int a, int i, int b) {
  if (S.mid >= 0 && lp == S.mid - 1) {
    cplx v = cz();
    const int rb = lrank(S, S.mid);
    for (int x = 0; x < rb; ++x) v = cfma(lentry(S, lp, a, i, x), lentry(S, S.mid, x, 0, b), v);
    return v;
  }
  if (S.lower && lp == S.D - 2) {
    cplx v = cz();
    const int rb = lrank(S, S.D - 1);
    for (int x = 0; x < rb; ++x) v = cfma(lentry(S, lp, a, i, x), lentry(S, S.D - 1, x, 0, 0), v);
    return v;
  }
  return lentry(S, lp, a, i, b);
}

__global__ void k_fft_store(StoreArgs S) {
  const int d = S.D - S.lower - (S.mid >= 0 ? 1 : 0);
  long long total = 0;
  for (int p = 0; p < d; ++p) total += (long long)S.cap[p] * 2 * S.cap[p + 1];
  for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < total;
       g += (long long)gridDim.x * blockDim.x) {
    int p = 0;
    while (p + 1 < d && g >= S.off[p + 1]) ++p;
    const int e = (int)(g - S.off[p]);
    const int c0 = (p == 0) ? 1 : obond(S, p);
    const int c1 = (p == d - 1) ? 1 : obond(S, p + 1);
    int o0 = c0, o1 = c1;
    if (S.realify) {
      o0 = (p == 0) ? 1 : 2 * c0;
      o1 = (p == d - 1) ? 1 : 2 * c1;
    }
    if (e >= o0 * 2 * o1) continue;
    const int A = e / (2 * o1), i = (e / o1) & 1, Bx = e % o1;
    const int lp = lcore(S, p);
    if (!S.realify) {
      const cplx v = centry(S, lp, A, i, Bx);
      static_cast<cplx*>(S.dst)[g] = v;
      continue;
    }
    const int s = A / c0, a = A - s * c0, tt = Bx / c1, b = Bx - tt * c1;
    const cplx z = centry(S, lp, a, i, b);
    double v;
    if (s == tt)
      v = z.x;
    else
      v = (s == 0) ? -z.y : z.y;
    if (S.kind == 0)
      static_cast<float*>(S.dst)[g] = (float)v;
    else
      static_cast<double*>(S.dst)[g] = v;
  }
  const long long g0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (g0 <= d) {
    const int j = (int)g0;
    int r = (j == 0 || j == d) ? 1 : obond(S, j);
    if (S.realify && j > 0 && j < d) r *= 2;
    S.dst_ranks[j] = r;
  }
}

// ------------------------------------------------------------------- host
static hipError_t g_attr_err = hipSuccess;
static std::once_flag g_attr_once;

static int set_attrs() {
  std::call_once(g_attr_once, [] {
    set_lds_limit(reinterpret_cast<const void*>(&k_qfft), (int)sizeof(Smem), &g_attr_err);
    set_lds_limit(reinterpret_cast<const void*>(&k_had_round), (int)sizeof(HadSmem),
                  &g_attr_err);
  });
  if (g_attr_err != hipSuccess) {
    set_hip_error(g_attr_err);
    return QTT_EHIP;
  }
  return QTT_OK;
}

struct Engine {
  cplx* cores;
  int32_t* ranks;
};

static Engine take_engine(Arena& ar, int D) {
  Engine e;
  e.cores = ar.take<cplx>((size_t)D * kSlot);
  e.ranks = ar.take<int32_t>((size_t)D + 1);
  return e;
}

struct LoadSpec {
  int core0 = 0;       // first engine core written
  int reverse = 0;
  int pad_mid = -1;    // source core before which a padding core goes, or -1
  int pad_end = 0;     // append a padding core
  int rotate = 0;      // swap the slices of the source's last core
  double scale = 1.0;
};

static int launch_load(const void* cores, int kind, const int32_t* src_ranks, const long long* off,
                       int d_src, Engine dst, const LoadSpec& sp, int32_t* status, hipStream_t s) {
  LoadArgs L;
  L.status = status;
  L.src = cores;
  L.kind = kind;
  L.src_ranks = src_ranks;
  for (int k = 0; k <= kMaxD; ++k) L.off[k] = k <= d_src ? off[k] : 0;
  L.d_src = d_src;
  L.dst = dst.cores;
  L.dst_ranks = dst.ranks;
  L.core0 = sp.core0;
  L.ncores = d_src + (sp.pad_mid >= 0 ? 1 : 0) + (sp.pad_end ? 1 : 0);
  L.reverse = sp.reverse;
  L.pad_mid = sp.pad_mid;
  L.pad_end = sp.pad_end;
  L.rotate = sp.rotate;
  L.scale = sp.scale;
  const long long total = (long long)L.ncores * kSlot;
  const int grid = (int)((total + 255) / 256);
  ProbeScope ps(QTT_K_OTHER, s);
  hipLaunchKernelGGL(k_fft_load, dim3(grid), dim3(256), 0, s, L);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

// element offsets of the cores of a caller's tensor
static void tensor_offsets(const qtt_tensor* t, long long* off) {
  long long o = 0;
  for (int k = 0; k <= t->d; ++k) {
    off[k] = o;
    if (k < t->d) o += (long long)t->cap[k] * 2 * t->cap[k + 1];
  }
}

static int load_tensor(const qtt_tensor* t, Engine dst, const LoadSpec& sp, int32_t* status,
                       hipStream_t s) {
  long long off[kMaxD + 1];
  tensor_offsets(t, off);
  const int kind = t->dtype == QTT_F32 ? 0 : (t->dtype == QTT_F64 ? 1 : 2);
  return launch_load(t->cores, kind, t->ranks, off, t->d, dst, sp, status, s);
}

static int launch_engine_load(Engine src, int D, Engine dst, int reverse, hipStream_t s) {
  long long off[kMaxD + 1];
  for (int k = 0; k <= D; ++k) off[k] = (long long)k * kSlot;
  LoadSpec sp;
  sp.reverse = reverse;
  return launch_load(src.cores, 2, src.ranks, off, D, dst, sp, nullptr, s);
}

static int launch_store(Engine src, int D, int reverse, int lower, int mid, int realify,
                        double scale, const qtt_tensor* y, hipStream_t s) {
  StoreArgs S;
  S.src = src.cores;
  S.src_ranks = src.ranks;
  S.D = D;
  S.reverse = reverse;
  S.lower = lower;
  S.mid = mid;
  S.realify = realify;
  S.scale = scale;
  S.dst = y->cores;
  S.kind = y->dtype == QTT_F32 ? 0 : (y->dtype == QTT_F64 ? 1 : 2);
  S.dst_ranks = y->ranks;
  const int d = y->d;
  long long o = 0;
  for (int k = 0; k <= kMaxD; ++k) {
    S.off[k] = o;
    S.cap[k] = k <= d ? y->cap[k] : 0;
    if (k < d) o += (long long)y->cap[k] * 2 * y->cap[k + 1];
  }
  const int grid = (int)std::min<long long>((o + 255) / 256 + 1, 4096);
  ProbeScope ps(QTT_K_OTHER, s);
  hipLaunchKernelGGL(k_fft_store, dim3(grid), dim3(256), 0, s, S);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

static int launch_qfft(const Task* tasks, int n, hipStream_t s) {
  int rc = set_attrs();
  if (rc) return rc;
  Tasks tt;
  tt.t[0] = tasks[0];
  tt.t[1] = n > 1 ? tasks[1] : tasks[0];
  ProbeScope ps(QTT_K_QFFT, s);
  hipLaunchKernelGGL(k_qfft, dim3(n), dim3(kNT), sizeof(Smem), s, tt);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

static Task make_task(Engine e, int32_t* status, int D, int sign, double eps, int max_rank,
                      double delta) {
  Task T;
  T.cores = e.cores;
  T.ranks = e.ranks;
  T.status = status;
  T.D = D;
  T.sign = sign;
  T.cap = max_rank > 0 ? max_rank : kR;
  T.lib_cap = max_rank > 0 ? 0 : 1;
  T.eps = eps;
  T.delta = delta;
  T.nblk = 1;
  T.lo[0] = 0;
  T.hi[0] = D;
  T.lo[1] = T.hi[1] = D;
  return T;
}

// the two axis blocks of an image: column digits (dx) then row digits
static void set_blocks(Task* T, int b0, int b1) {
  T->nblk = 2;
  T->lo[0] = 0;
  T->hi[0] = b0;
  T->lo[1] = b0;
  T->hi[1] = b0 + b1;
}

// the rank bound of a transform's output: min(2^k, 2^(D-k), cap)
static void fft_caps(int D, int cap, int32_t* out) {
  for (int k = 0; k <= D; ++k) {
    long long c = cap;
    c = std::min<long long>(c, 1LL << std::min(k, 40));
    c = std::min<long long>(c, 1LL << std::min(D - k, 40));
    out[k] = (k == 0 || k == D) ? 1 : (int32_t)c;
  }
}

static bool rule_ok(double eps, int max_rank, double delta) {
  return eps >= 0.0 && isfinite(eps) && delta >= 0.0 && delta < 1.0 && max_rank >= 0 &&
         max_rank <= kR;
}

static int tensor_in_ok(const qtt_tensor* t, int dtype_lo, int dtype_hi) {
  if (!t || t->d < 1 || t->d > kMaxD || t->dtype < dtype_lo || t->dtype > dtype_hi || !t->ranks ||
      !t->cores)
    return QTT_EINVAL;
  if (t->cap[0] != 1 || t->cap[t->d] != 1) return QTT_EINVAL;
  for (int k = 1; k < t->d; ++k)
    if (t->cap[k] < 1) return QTT_EINVAL;
  return QTT_OK;
}

static size_t fft_ws(int D) {
  Arena ar(nullptr);
  take_engine(ar, D);
  return ar.size();
}

static size_t conv_fft_ws(int D) {
  Arena ar(nullptr);
  for (int i = 0; i < 4; ++i) take_engine(ar, D);
  ar.take<cplx>((size_t)(D + 1) * kHad * kL);
  ar.take<cplx>((size_t)2 * kHad * kL);
  ar.take<cplx>((size_t)2 * kL * kR * kR);
  ar.take<cplx>((size_t)kL * kHad);
  return ar.size();
}

}  // namespace fftq
}  // namespace qtt

using namespace qtt;
using namespace qtt::fftq;

extern "C" {

int qtt_query_fft(int d, int max_rank, int32_t* cap, size_t* ws_bytes) {
  if (d < 1 || d > kMaxD || max_rank < 0 || max_rank > kR) return QTT_EINVAL;
  if (cap) fft_caps(d, max_rank > 0 ? max_rank : kR, cap);
  if (ws_bytes) *ws_bytes = fft_ws(d);
  return QTT_OK;
}

int qtt_fft(const qtt_tensor* x, int inverse, double eps, int max_rank, double delta, qtt_tensor* y,
            void* ws, size_t ws_bytes, void* stream) {
  int rc = tensor_in_ok(x, QTT_C128, QTT_C128);
  if (rc) return rc;
  if (!rule_ok(eps, max_rank, delta)) return QTT_EINVAL;
  const int D = x->d;
  if (!y || y->d != D || y->dtype != QTT_C128 || !y->ranks || !y->cores) return QTT_EINVAL;
  int32_t need[kMaxD + 1];
  fft_caps(D, max_rank > 0 ? max_rank : kR, need);
  for (int k = 0; k <= D; ++k)
    if (y->cap[k] < need[k]) return QTT_ENOSPC;
  if (!ws || ws_bytes < fft_ws(D)) return QTT_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena ar(ws);
  Engine e = take_engine(ar, D);
  LoadSpec sp;
  sp.reverse = inverse ? 1 : 0;
  rc = load_tensor(x, e, sp, y->status, s);
  if (rc) return rc;
  const Task T = make_task(e, y->status, D, inverse ? 1 : -1, eps, max_rank, delta);
  rc = launch_qfft(&T, 1, s);
  if (rc) return rc;
  return launch_store(e, D, inverse ? 1 : 0, 0, -1, 0, inverse ? ldexp(1.0, -D) : 1.0, y, s);
}

static int axes_ok(int d, int n_axes, const int32_t* axis_modes) {
  if (n_axes == 1) return (!axis_modes || axis_modes[0] == d) ? QTT_OK : QTT_EINVAL;
  if (n_axes != 2 || !axis_modes) return QTT_EINVAL;
  if (axis_modes[0] < 1 || axis_modes[1] < 1 || axis_modes[0] + axis_modes[1] != d)
    return QTT_EINVAL;
  return QTT_OK;
}

// capacities of the output: the inverse transform's bond bound (doubled by
// the real part) on the bonds that remain once the padding digits are gone
static void conv_fft_caps(int d, int n_axes, const int32_t* axis_modes, int R, int32_t* y_cap) {
  const int D = d + n_axes;
  int32_t c[kMaxD + 1];
  fft_caps(D, R, c);
  const int mid = n_axes == 2 ? axis_modes[0] : -1;  // engine core of the column padding
  for (int j = 0; j <= d; ++j) {
    const int lj = j + ((mid >= 0 && j >= mid) ? 1 : 0);
    y_cap[j] = (j == 0 || j == d) ? 1 : 2 * c[lj];
  }
}

int qtt_query_conv_fft(int d, int n_axes, const int32_t* axis_modes, int max_rank_hat,
                       int oversample, int32_t* y_cap, size_t* ws_bytes) {
  if (d < 1 || d + n_axes > kMaxD || max_rank_hat < 1 || max_rank_hat > kR || oversample < 0 ||
      max_rank_hat + oversample > kL)
    return QTT_EINVAL;
  if (axes_ok(d, n_axes, axis_modes)) return QTT_EINVAL;
  if (y_cap) conv_fft_caps(d, n_axes, axis_modes, max_rank_hat, y_cap);
  if (ws_bytes) *ws_bytes = conv_fft_ws(d + n_axes);
  return QTT_OK;
}

int qtt_conv_fft(const qtt_tensor* f, const qtt_tensor* w, int n_axes, const int32_t* axis_modes,
                 double eps_hat, int max_rank_hat, double delta_hat, int oversample,
                 uint64_t seed, qtt_tensor* y, void* ws, size_t ws_bytes, void* stream) {
  int rc = tensor_in_ok(f, QTT_F32, QTT_F64);
  if (rc) return rc;
  if (!w || (n_axes != 1 && n_axes != 2)) return QTT_EINVAL;
  const int d = f->d, D = d + n_axes;
  if (D > kMaxD) return QTT_ENOTSUP;
  if (axes_ok(d, n_axes, axis_modes)) return QTT_EINVAL;
  for (int a = 0; a < n_axes; ++a) {
    rc = tensor_in_ok(&w[a], QTT_F32, QTT_F64);
    if (rc) return rc;
    const int need = (n_axes == 1 ? d : axis_modes[a]) + 1;
    if (w[a].d != need) return QTT_EINVAL;
  }
  if (!rule_ok(eps_hat, max_rank_hat, delta_hat) || max_rank_hat < 1 || oversample < 0 ||
      max_rank_hat + oversample > kL)
    return QTT_EINVAL;
  if (!y || y->d != d || y->dtype != f->dtype || !y->ranks || !y->cores) return QTT_EINVAL;
  if (y->cap[0] != 1 || y->cap[d] != 1) return QTT_EINVAL;
  int32_t need[kMaxD + 1];
  conv_fft_caps(d, n_axes, axis_modes, max_rank_hat, need);
  for (int k = 0; k <= d; ++k)
    if (y->cap[k] < need[k]) return QTT_ENOSPC;
  if (!ws || ws_bytes < conv_fft_ws(D)) return QTT_ENOSPC;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Arena ar(ws);
  Engine ef = take_engine(ar, D), eg = take_engine(ar, D), eh = take_engine(ar, D),
         er = take_engine(ar, D);
  cplx* W = ar.take<cplx>((size_t)(D + 1) * kHad * kL);
  cplx* Mb = ar.take<cplx>((size_t)2 * kHad * kL);
  cplx* T1 = ar.take<cplx>((size_t)2 * kL * kR * kR);
  cplx* Zb = ar.take<cplx>((size_t)kL * kHad);
  const int dx = n_axes == 2 ? axis_modes[0] : d;
  // data: a padding digit after each axis
  LoadSpec sf;
  sf.pad_mid = n_axes == 2 ? dx : -1;
  sf.pad_end = 1;
  rc = load_tensor(f, ef, sf, y->status, s);
  if (rc) return rc;
  // kernel: the rotated generator of each axis, one after the other
  for (int a = 0; a < n_axes; ++a) {
    LoadSpec sw;
    sw.core0 = a == 0 ? 0 : dx + 1;
    sw.rotate = 1;
    rc = load_tensor(&w[a], eg, sw, y->status, s);
    if (rc) return rc;
  }
  Task tk[2] = {make_task(ef, y->status, D, -1, eps_hat, max_rank_hat, delta_hat),
                make_task(eg, y->status, D, -1, eps_hat, max_rank_hat, delta_hat)};
  if (n_axes == 2) {
    set_blocks(&tk[0], dx + 1, D - dx - 1);
    set_blocks(&tk[1], dx + 1, D - dx - 1);
  }
  rc = launch_qfft(tk, 2, s);
  if (rc) return rc;
  HadArgs H;
  H.A = ef.cores;
  H.ra = ef.ranks;
  H.Bm = eg.cores;
  H.rb = eg.ranks;
  H.out = make_task(eh, y->status, D, 1, eps_hat, max_rank_hat, delta_hat);
  H.W = W;
  H.Mb = Mb;
  H.T1 = T1;
  H.Zb = Zb;
  H.ell = max_rank_hat + oversample;
  H.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
  H.k1 = (uint32_t)(seed >> 32);
  {
    rc = set_attrs();
    if (rc) return rc;
    ProbeScope ps(QTT_K_QFFT_HADAMARD, s);
    hipLaunchKernelGGL(k_had_round, dim3(1), dim3(kNT), sizeof(HadSmem), s, H);
    QTT_LAUNCH_CHECK();
  }
  // QiFFT: reversing restores the digit order inside each axis and mirrors
  // the axes; the forward stages with the +1 exponent run on the mirrored
  // blocks and the result is reversed back
  rc = launch_engine_load(eh, D, er, 1, s);
  if (rc) return rc;
  Task ti = make_task(er, y->status, D, 1, eps_hat, max_rank_hat, delta_hat);
  if (n_axes == 2) set_blocks(&ti, D - dx - 1, dx + 1);
  rc = launch_qfft(&ti, 1, s);
  if (rc) return rc;
  return launch_store(er, D, 1, 1, n_axes == 2 ? dx : -1, 1, ldexp(1.0, -D), y, s);
}

}  // extern "C"

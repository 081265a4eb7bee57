// One-workgroup FP64 symmetric eigensolver and the truncation rule.
//
// Every truncated SVD of the TT-SVD sweep (Algorithm 1) is taken through the
// Gram matrix G = X^T X of the unfolding (or the dual X X^T when it is
// smaller): G = U diag(sigma^2) U^T.  The eigensolver is the cyclic Jacobi
// method with the parallel "circle" ordering: each round applies n/2
// disjoint plane rotations, and the whole workgroup updates the rotated
// matrix in 2x2 blocks (block (s,t) <- J_s^T A_st J_t), so a round costs two
// barriers.  Sweeps repeat until no off-diagonal entry is above
// 1e-15 * sqrt(|a_pp a_qq|) (or an absolute floor set by the trace).
#pragma once

#include "qtt_internal.hpp"

namespace qtt {

// pair t of round r in the circle schedule for n (even) indices
// (r, t < n-1, so the residues need one conditional subtraction)
__device__ __forceinline__ void jpair(int r, int t, int n, int& p, int& q) {
  const int m = n - 1;
  if (t == 0) {
    p = m;
    q = r;
  } else {
    p = r + t;
    if (p >= m) p -= m;
    q = r - t;
    if (q < 0) q += m;
  }
}

// Plane rotation (c, s) that zeroes a_pq of the symmetric 2x2 block
// [[app, apq], [apq, aqq]] with J = [[c, s], [-s, c]] (J^T A J diagonal),
// tangent of the smaller angle (Golub & Van Loan, symmetric Schur 2x2).
__device__ __forceinline__ void jrot(double app, double aqq, double apq, double& c, double& s) {
  const double theta = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(theta) > 1e150) {
    t = 0.5 / theta;
  } else {
    t = 1.0 / (fabs(theta) + sqrt(fma(theta, theta, 1.0)));
    if (theta < 0.0) t = -t;
  }
  c = 1.0 / sqrt(fma(t, t, 1.0));
  s = t * c;
}

// A: E x E symmetric (row stride lda >= E+1, E+1 rows allocated when E is odd).
// On return diag(A) = eigenvalues, columns of V = eigenvectors (stride lda).
// cs: >= 2*(E/2+1) doubles of shared scratch; pq: >= 2*(E/2+1) ints of
// shared scratch; flag: one shared int.
template <int NT>
__device__ int jacobi_eig(double* A, double* V, int E, int lda, double* cs, int* pq, int* flag) {
  const int tid = threadIdx.x;
  const int n = E + (E & 1);
  const int np = n / 2;
  if (E & 1) {
    for (int i = tid; i < n; i += NT) {
      A[E * lda + i] = 0.0;
      A[i * lda + E] = 0.0;
    }
  }
  for (int idx = tid; idx < n * n; idx += NT) {
    const int r = idx / n, c = idx - r * n;
    V[r * lda + c] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (n < 2) return 0;
  double tr = 0.0;
  for (int i = 0; i < E; ++i) tr += fabs(A[i * lda + i]);
  // pairs coupled below 1e-18 of the trace are left alone: their rotation
  // would only move rounding noise (eigenvalues below that level are not
  // resolved by a Gram matrix anyway)
  const double floor_abs = 1e-300 + 1e-18 * tr;
  const double tol = 1e-15;
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      if (tid < np) {
        int p, q;
        jpair(r, tid, n, p, q);
        const double app = A[p * lda + p], aqq = A[q * lda + q], apq = A[p * lda + q];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > floor_abs && fabs(apq) > tol * sqrt(fabs(app * aqq))) {
          jrot(app, aqq, apq, c, s);
          *flag = 1;
        }
        cs[2 * tid] = c;
        cs[2 * tid + 1] = s;
        pq[2 * tid] = p;
        pq[2 * tid + 1] = q;
      }
      __syncthreads();
      for (int b = tid; b < np * np; b += NT) {
        const int sI = b / np, tI = b - sI * np;
        const double sS = cs[2 * sI + 1], sT = cs[2 * tI + 1];
        if (sS == 0.0 && sT == 0.0) continue;  // both rotations are the identity
        const double cS = cs[2 * sI], cT = cs[2 * tI];
        const int ps = pq[2 * sI], qs = pq[2 * sI + 1];
        const int pt = pq[2 * tI], qt = pq[2 * tI + 1];
        const double a11 = A[ps * lda + pt], a12 = A[ps * lda + qt];
        const double a21 = A[qs * lda + pt], a22 = A[qs * lda + qt];
        // columns pt, qt: (x, y) -> (c x - s y, s x + c y)
        const double b11 = cT * a11 - sT * a12, b12 = sT * a11 + cT * a12;
        const double b21 = cT * a21 - sT * a22, b22 = sT * a21 + cT * a22;
        // rows ps, qs: (x, y) -> (c x - s y, s x + c y)
        double n11 = cS * b11 - sS * b21, n12 = cS * b12 - sS * b22;
        double n21 = sS * b11 + cS * b21, n22 = sS * b12 + cS * b22;
        if (sI == tI) {  // the rotated 2x2 block is diagonal
          n12 = 0.0;
          n21 = 0.0;
        }
        A[ps * lda + pt] = n11;
        A[ps * lda + qt] = n12;
        A[qs * lda + pt] = n21;
        A[qs * lda + qt] = n22;
        if (sT != 0.0) {
          const double v11 = V[ps * lda + pt], v12 = V[ps * lda + qt];
          const double v21 = V[qs * lda + pt], v22 = V[qs * lda + qt];
          V[ps * lda + pt] = cT * v11 - sT * v12;
          V[ps * lda + qt] = sT * v11 + cT * v12;
          V[qs * lda + pt] = cT * v21 - sT * v22;
          V[qs * lda + qt] = sT * v21 + cT * v22;
        }
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (f == 0) break;
  }
  return sweep + 1;
}

// ------------------------------------------------------ 32-lane reductions
// Butterfly sum over a group of 32 lanes: DPP quad permutes (xor 1, xor 2),
// half-row and row mirrors (sums over 8 and 16 lanes), then a swizzle with
// xor 16.  Every lane of the group ends with the group sum.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double swz16_d(double x) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(x), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(x), 0x401F);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double sum32(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  v += swz16_d(v);       // lane ^ 16
  return v;
}

__device__ __forceinline__ double sum16(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

// 1/sqrt(x) to FP64 accuracy: hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_acc(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}

// Eigendecomposition of a symmetric positive semidefinite Gram matrix G
// (E x E in A, row stride lda) through its Cholesky factor and a one-sided
// Jacobi sweep (Hestenes):
//   1. G + delta I = L L^T (left-looking Cholesky, one 16-lane group per row;
//      delta starts at 1e-14 trace(G) and grows 16x until every pivot is
//      positive -- the shift moves every eigenvalue by delta and leaves the
//      eigenvectors unchanged); column j of L is stored as row j of A;
//   2. the columns l_j are orthogonalised by plane rotations, L V = W, until
//      (l_p.l_q)^2 <= 1e-30 |l_p|^2 |l_q|^2 or |l_p.l_q| <= 1e-18 trace(G) for
//      all pairs (circle ordering, one 32-lane group per pair, one barrier
//      per round).  The tangent only steers the angle (approximate
//      reciprocals); c = 1/sqrt(1+t^2) is exact to rounding so every rotation
//      is orthogonal;
//   3. G + delta I = W W^T: eigenvectors w_j/|w_j|, eigenvalues |w_j|^2 - delta.
// On return the columns of V (stride lda) are the eigenvectors and lam_raw[j]
// the eigenvalue of column j (unsorted).  V's buffer holds a copy of G for
// the Cholesky retries.  Returns the number of sweeps.
template <int NT>
__device__ int gram_eig(double* A, double* V, int E, int lda, double* lam_raw, double* red,
                        int* flag, int* tim = nullptr) {
  const int tid = threadIdx.x;
  const int lane = tid & 31, grp = tid >> 5;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG = NT / 32, NG16 = NT / 16;
  (void)red;
#ifdef QTT_EIG_TIMING
  const long long c0 = wall_clock64();
#endif
  for (int e = tid; e < E * E; e += NT) {
    const int i = e / E, j = e - i * E;
    V[i * lda + j] = A[i * lda + j];
  }
  __syncthreads();
  double tr = 0.0;
  for (int i = 0; i < E; ++i) tr += fabs(V[i * lda + i]);
  double delta = 1e-14 * tr + 1e-300;
  // ---- 1. left-looking Cholesky of G + delta I:  A[j][i] = L[i][j]
  for (int attempt = 0; attempt < 12; ++attempt) {
    for (int e = tid; e < (E + 1) * lda; e += NT) A[e] = 0.0;
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int j = 0; j < E; ++j) {
      // s_i = G[i][j] + delta[i==j] - sum_{c<j} L[i][c] L[j][c],  i >= j
      for (int i = j + g16; i < E; i += NG16) {
        double s = 0.0;
        for (int c = l16; c < j; c += 16) s = fma(A[c * lda + i], A[c * lda + j], s);
        s = sum16(s);
        if (l16 == 0) lam_raw[i] = V[i * lda + j] + (i == j ? delta : 0.0) - s;
      }
      __syncthreads();
      const double d = lam_raw[j];
      if (d <= 0.0) {
        if (tid == 0) *flag = 1;
        break;  // uniform: every thread read the same pivot
      }
      const double inv = rsqrt_acc(d);
      for (int i = j + tid; i < E; i += NT) A[j * lda + i] = (i == j) ? d * inv : lam_raw[i] * inv;
      __syncthreads();
    }
    __syncthreads();
    const int failed = *flag;
    __syncthreads();
    if (!failed) break;
    delta *= 16.0;
  }
  const double gfloor = 1e-18 * tr + 1e-300;
#ifdef QTT_EIG_TIMING
  const long long c1 = wall_clock64();
#endif
  // ---- 2. one-sided Jacobi on the columns of L (rows of A)
  const int n = E + (E & 1);  // row E of A is zero when E is odd
  const int np = n / 2;
  int sweep = 0;
  for (; sweep < 40 && n >= 2; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      for (int t = grp; t < np; t += NG) {
        int pp, qq;
        jpair(r, t, n, pp, qq);
        double* xp = A + pp * lda;
        double* xq = A + qq * lda;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = lane; i < E; i += 32) {
          const double x = xp[i], y = xq[i];
          a = fma(x, x, a);
          b = fma(y, y, b);
          g = fma(x, y, g);
        }
        a = sum32(a);
        b = sum32(b);
        g = sum32(g);
        if (g * g > 1e-30 * a * b && fabs(g) > gfloor) {
          // tangent of the smaller rotation angle (steering only)
          double zeta = (b - a) * 0.5 * __builtin_amdgcn_rcp(g);
          zeta = fmax(fmin(zeta, 1e30), -1e30);
          const float zf = (float)zeta;
          float tf = __builtin_amdgcn_rcpf(fabsf(zf) + __builtin_amdgcn_sqrtf(fmaf(zf, zf, 1.0f)));
          if (zf < 0.0f) tf = -tf;
          const double t = (double)tf;
          const double c = rsqrt_acc(fma(t, t, 1.0));
          const double s = t * c;
          for (int i = lane; i < E; i += 32) {
            const double x = xp[i], y = xq[i];
            xp[i] = c * x - s * y;
            xq[i] = s * x + c * y;
          }
          if (lane == 0) *flag = 1;
        }
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (f == 0) break;
  }
#ifdef QTT_EIG_TIMING
  const long long c2 = wall_clock64();
#endif
  // ---- 3. eigenpairs: w_j = row j of A
  for (int j = grp; j < E; j += NG) {
    const double* w = A + j * lda;
    double a = 0.0;
    for (int i = lane; i < E; i += 32) a = fma(w[i], w[i], a);
    a = sum32(a);
    const double inv = a > 0.0 ? rsqrt_acc(a) : 0.0;
    for (int i = lane; i < E; i += 32) V[i * lda + j] = w[i] * inv;
    if (lane == 0) lam_raw[j] = a - delta;
  }
  __syncthreads();
#ifdef QTT_EIG_TIMING
  const long long c3 = wall_clock64();
  if (tid == 0 && tim) {
    tim[0] = (int)(c1 - c0);
    tim[1] = (int)(c2 - c1);
    tim[2] = (int)(c3 - c2);
    tim[3] = E;
  }
#else
  (void)tim;
#endif
  return sweep + 1;
}

// Sort lam_raw[0..E) in non-increasing order: lam[pos] = value, perm[pos] = index.
template <int NT>
__device__ void sort_vals(const double* lam_raw, int E, double* lam, int* perm, int finite) {
  const int tid = threadIdx.x;
  for (int i = tid; i < E; i += NT) {
    if (!finite) {
      lam[i] = 0.0;
      perm[i] = i;
      continue;
    }
    const double li = lam_raw[i];
    int pos = 0;
    for (int j = 0; j < E; ++j) {
      const double lj = lam_raw[j];
      pos += (lj > li) || (lj == li && j < i);
    }
    lam[pos] = li;
    perm[pos] = i;
  }
}

// Sort diag(A) in non-increasing order: lam[pos] = value, perm[pos] = index.
// A non-finite diagonal leaves the identity order with zero values.
template <int NT>
__device__ void sort_eigs(const double* A, int lda, int E, double* lam, int* perm, int finite) {
  const int tid = threadIdx.x;
  for (int i = tid; i < E; i += NT) {
    if (!finite) {
      lam[i] = 0.0;
      perm[i] = i;
      continue;
    }
    const double li = A[i * lda + i];
    int pos = 0;
    for (int j = 0; j < E; ++j) {
      const double lj = A[j * lda + j];
      pos += (lj > li) || (lj == li && j < i);
    }
    lam[pos] = li;
    perm[pos] = i;
  }
}

// Algorithm 1's rule on the sorted eigenvalues of the Gram matrix: smallest
// r >= 1 with sum_{i >= r} lam_i <= tau2 (tails summed from the small end),
// then min(r, cap).  *over is set when the eps-rank exceeded cap.
__device__ inline int truncation_rank_dev(const double* lam, int E, double tau2, int cap,
                                          int* over) {
  double tail = 0.0;
  int r = E;
  for (int i = E - 1; i >= 1; --i) {
    const double l = lam[i] > 0.0 ? lam[i] : 0.0;
    const double t2 = tail + l;
    if (t2 <= tau2) {
      tail = t2;
      r = i;
    } else {
      break;
    }
  }
  if (r < 1) r = 1;
  *over = r > cap;
  return r < cap ? r : cap;
}

}  // namespace qtt

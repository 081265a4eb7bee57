// One-workgroup FP64 symmetric eigensolver for the Gram matrices of the
// TT-SVD sweep (Algorithm 1): every truncated SVD is taken through
// G = X^T X = U diag(sigma^2) U^T.
//
//   1. Householder tridiagonalisation G = Q T Q^T (the reflector of step j
//      annihilates column j below the subdiagonal; two barriers per step);
//      for orders up to 64 Q^T is accumulated alongside in registers;
//   2. eigenvalues of T by parallel multisection with Sturm counts (sign
//      changes of the leading principal minors of T - x I): a lane group
//      brackets one eigenvalue and narrows it (G+1)-fold per pass, to a
//      width of about 1e-16 ||T||; when the rank cap binds only the cap
//      largest are computed;
//   3. the caller picks the rank from the eigenvalues;
//   4. eigenvectors of T for the kept eigenvalues only by a twisted
//      factorisation of T - lambda I (top-down and bottom-up LDL^T sweeps;
//      the twist index minimises |gamma_r|), then orthonormalised: one
//      Newton-Schulz step on the matrix cores when they are orthonormal to
//      first order, modified Gram-Schmidt otherwise;
//   5. back-transformation U = Q Z (one matrix-core product for orders up to
//      64, the stored reflectors above).
// Orders up to 64 work on LDS arrays of one workgroup; larger ones keep A and
// V in global scratch.
#pragma once

#include "qtt_internal.hpp"

namespace qtt {

// ---------------------------------------------------------- lane reductions
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  // every lane reads a valid lane under the patterns used here, so no old
  // value is needed (mov_dpp, not update_dpp: no register initialisation)
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// sum over the 16 lanes of a DPP row (all lanes of the row get the sum)
__device__ __forceinline__ double sum16(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}
// x[l % 32] + x[l % 32 + 32] in every lane l (the two half waves swap)
__device__ __forceinline__ double sum_halves(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
// x + (x of the neighbouring DPP row): rows 0+1 and 2+3 paired
__device__ __forceinline__ double sum_row_pairs(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}
// sum over the 32 lanes of a half wave
__device__ __forceinline__ double sum32(double v) { return sum_row_pairs(sum16(v)); }
// sum over the whole wave (every lane gets the sum)
__device__ __forceinline__ double sum64(double v) { return sum_halves(sum_row_pairs(sum16(v))); }
// x summed over the four DPP rows at the same position, in every lane
__device__ __forceinline__ double sum_rows4(double x) { return sum_halves(sum_row_pairs(x)); }

// max over the whole wave of non-negative values (every lane gets it)
__device__ __forceinline__ double max64(double v) {
  v = fmax(v, dpp_d<0xB1>(v));
  v = fmax(v, dpp_d<0x4E>(v));
  v = fmax(v, dpp_d<0x141>(v));
  v = fmax(v, dpp_d<0x140>(v));
  {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const auto a16 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b16 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    v = fmax(__hiloint2double(b16[0], a16[0]), __hiloint2double(b16[1], a16[1]));
  }
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto a32 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto b32 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return fmax(__hiloint2double(b32[0], a32[0]), __hiloint2double(b32[1], a32[1]));
}

// Gershgorin bound max_i |a_i| + |b_{i-1}| + |b_i| of the tridiagonal T,
// by wave 0 and handed to every thread through slot (one double of LDS).
__device__ inline double tridiag_gersh(lds_ptr<const double> dg, lds_ptr<const double> od, int E,
                                       ldsd slot) {
  if (threadIdx.x < 64) {
    double m = 0.0;
    for (int i = threadIdx.x; i < E; i += 64)
      m = fmax(m, fabs(dg[i]) + (i > 0 ? fabs(od[i - 1]) : 0.0) + (i + 1 < E ? fabs(od[i]) : 0.0));
    m = max64(m);
    if (threadIdx.x == 0) slot[0] = m;
  }
  __syncthreads();
  return slot[0];
}

// 1/x to FP64 accuracy from the hardware estimate (two Newton steps)
__device__ __forceinline__ double rcp_acc(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * fma(-x, y, 2.0);
  y = y * fma(-x, y, 2.0);
  return y;
}

// 1/sqrt(x) to FP64 accuracy from the hardware estimate (two Newton steps)
__device__ __forceinline__ double rsq_acc(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * fma(-hx * y, y, 1.5);
  y = y * fma(-hx * y, y, 1.5);
  return y;
}

// ------------------------------------------------------- tridiagonalisation
// A (E x E symmetric, full storage, stride lda >= 16*BS, at least 16*BS
// rows allocated, E <= 16*BS) -> T (dg, od)
// and reflectors.  The matrix is held in registers: thread (br, bc) =
// (tid / 16, tid % 16) owns the BS x BS block at rows br*BS.., columns
// bc*BS.., so the 16 owners of a block row are one DPP row of a wave.  Step
// j applies H_j = I - beta_j v v^T (v zero in entries 0..j) to the whole
// matrix, A <- H A H, as A - v w^T - w v^T with p = beta A v and
// w = p - (beta/2)(p.v) v; rows and columns 0..j-1 stay untouched because
// v vanishes there and A is already reduced there.  v_j is left in
// A[j+1.., j] (LDS) and beta_j in bt[j].  buf: >= 4*kMaxM doubles (double-
// buffered column and p vectors, so two barriers per step suffice).
template <int NT, int BS, class MP>
__device__ void sy_tridiag(MP A, int E, int lda, ldsd dg, ldsd od, ldsd bt, ldsd buf) {
  static_assert(NT == 256, "16 x 16 thread grid");
  const int tid = threadIdx.x;
  const int br = tid >> 4, bc = tid & 15;
  const int l64 = tid & 63;
  const int r0 = br * BS, c0 = bc * BS;
  double a[BS][BS];
#pragma unroll
  for (int ii = 0; ii < BS; ++ii)
#pragma unroll
    for (int cc = 0; cc < BS; ++cc) {
      const int r = r0 + ii, c = c0 + cc;
      const double t = A[r * lda + c];  // r, c < 16*BS <= lda: in bounds
      a[ii][cc] = (r < E && c < E) ? t : 0.0;
    }
  __syncthreads();  // A (LDS) now only receives reflectors
  for (int j = 0; j + 2 < E; ++j) {
    ldsd colb = buf + (j & 1) * (2 * kMaxM);
    ldsd pb = colb + kMaxM;
    // 1. publish column j
    if (bc == j / BS) {
      const int jc = j - c0;
#pragma unroll
      for (int ii = 0; ii < BS; ++ii) {
        double v = a[ii][0];
#pragma unroll
        for (int cc = 1; cc < BS; ++cc) v = (jc == cc) ? a[ii][cc] : v;
        colb[r0 + ii] = v;  // rows >= E hold zeros
      }
    }
    __syncthreads();
    // 2. reflector (every wave, redundantly); loads are unconditional (the
    // buffers hold 16*BS <= kMaxM entries) and masked afterwards
    double xs = 0.0;
#pragma unroll
    for (int h = 0; h < BS / 4; ++h) {
      const int i = l64 + 64 * h;
      const double t = colb[i];
      xs = (i > j && i < E) ? fma(t, t, xs) : xs;
    }
    xs = sum64(xs);
    const double x0 = colb[j + 1];
    double vc[BS], cr[BS];
#pragma unroll
    for (int cc = 0; cc < BS; ++cc) vc[cc] = colb[c0 + cc];
#pragma unroll
    for (int ii = 0; ii < BS; ++ii) cr[ii] = colb[r0 + ii];
    if (xs - x0 * x0 <= 1e-300 + 1e-32 * xs) {  // column already reduced (uniform)
      if (tid == 0) {
        bt[j] = 0.0;
        od[j] = x0;
      }
      if (br == j / BS && bc == j / BS) {
        const int jj = j - r0;
#pragma unroll
        for (int ii = 0; ii < BS; ++ii)
          if (ii == jj) dg[j] = a[ii][ii];
      }
      continue;
    }
    const double alpha = sqrt(xs);
    const double sg = x0 >= 0.0 ? 1.0 : -1.0;
    const double v0 = x0 + sg * alpha;
    const double beta = 2.0 / (xs - x0 * x0 + v0 * v0);
    // 3. p = beta A v: partial over the own columns, summed over the block row
#pragma unroll
    for (int cc = 0; cc < BS; ++cc) {
      const int c = c0 + cc;
      vc[cc] = (c <= j || c >= E) ? 0.0 : (c == j + 1 ? v0 : vc[cc]);
    }
    double vr[BS];
#pragma unroll
    for (int ii = 0; ii < BS; ++ii) {
      const int r = r0 + ii;
      vr[ii] = (r <= j || r >= E) ? 0.0 : (r == j + 1 ? v0 : cr[ii]);
    }
    double pp[BS];
#pragma unroll
    for (int ii = 0; ii < BS; ++ii) {
      double t0 = 0.0, t1 = 0.0;
#pragma unroll
      for (int cc = 0; cc < BS; cc += 2) {
        t0 = fma(a[ii][cc], vc[cc], t0);
        t1 = fma(a[ii][cc + 1], vc[cc + 1], t1);
      }
      pp[ii] = t0 + t1;
    }
#pragma unroll
    for (int ii = 0; ii < BS; ++ii) pp[ii] = sum16(pp[ii]);
    if (bc == 0) {
#pragma unroll
      for (int ii = 0; ii < BS; ++ii) pb[r0 + ii] = beta * pp[ii];
    }
    // reflector storage and the diagonal entry (unchanged by this step)
    if (tid < 64) {
#pragma unroll
      for (int h = 0; h < BS / 4; ++h) {
        const int i = l64 + 64 * h;
        if (i > j && i < E) A[i * lda + j] = (i == j + 1) ? v0 : colb[i];
      }
    }
    if (br == j / BS && bc == j / BS) {
      const int jj = j - r0;
#pragma unroll
      for (int ii = 0; ii < BS; ++ii)
        if (ii == jj) dg[j] = a[ii][ii];
    }
    if (tid == 0) {
      od[j] = -sg * alpha;
      bt[j] = beta;
    }
    __syncthreads();
    // 4. K = beta/2 p.v ; w = p - K v on own rows and columns
    double pv = 0.0;
#pragma unroll
    for (int h = 0; h < BS / 4; ++h) {
      const int i = l64 + 64 * h;
      const double pi = pb[i], ci = colb[i];
      pv = (i > j && i < E) ? fma(pi, (i == j + 1) ? v0 : ci, pv) : pv;
    }
    const double K = 0.5 * beta * sum64(pv);
    double wr[BS], wc[BS];
#pragma unroll
    for (int ii = 0; ii < BS; ++ii) wr[ii] = pb[r0 + ii];
#pragma unroll
    for (int cc = 0; cc < BS; ++cc) wc[cc] = pb[c0 + cc];
#pragma unroll
    for (int ii = 0; ii < BS; ++ii) wr[ii] = (r0 + ii < E) ? fma(-K, vr[ii], wr[ii]) : 0.0;
#pragma unroll
    for (int cc = 0; cc < BS; ++cc) wc[cc] = (c0 + cc < E) ? fma(-K, vc[cc], wc[cc]) : 0.0;
    // 5. rank-2 update
#pragma unroll
    for (int ii = 0; ii < BS; ++ii)
#pragma unroll
      for (int cc = 0; cc < BS; ++cc)
        a[ii][cc] = fma(-vr[ii], wc[cc], fma(-wr[ii], vc[cc], a[ii][cc]));
  }
  // trailing 2 x 2 block
  const int jl = E - 2;
#pragma unroll
  for (int ii = 0; ii < BS; ++ii)
#pragma unroll
    for (int cc = 0; cc < BS; ++cc) {
      const int r = r0 + ii, c = c0 + cc;
      if (E >= 2 && r == jl + 1 && c == jl) od[jl] = a[ii][cc];
      if (r == c && r >= jl && r < E && r >= 0) dg[r] = a[ii][cc];
    }
  if (tid == 0) {
    if (E >= 2) bt[E - 2] = 0.0;
    bt[E - 1] = 0.0;
  }
  __syncthreads();
}

// Tridiagonalisation for E <= 64, four waves.  Wave q holds rows
// 16q..16q+15 of A in registers, lane c column c, so the product A v needs no
// exchange inside a wave (each wave multiplies its 16 rows; the four partial
// vectors meet in LDS), and the step loop is unrolled by 16 so that row j,
// published at step j, is a register with a compile-time index.  Same
// reflectors as sy_tridiag (H_j = I - beta_j v v^T, v_{j+1} = x0 + sign(x0)
// alpha).  The product X = H_{E-3} ... H_0 = Q^T is accumulated alongside in
// the same register layout (its update needs vT X, one more partial vector
// per wave in the same LDS exchange) and left in A; beta_j in bt[j].
// A: >= 64 rows allocated, lda >= 64.  buf: >= 960 doubles.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Sixteen consecutive doubles from 16-byte aligned LDS as eight 128-bit
// loads: their 16-bit immediate offsets reach every buffer of the solver from
// one base register, where pairs of 64-bit loads needed an address add each.
typedef double lds_d2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void lds_load16(lds_ptr<const double> p, double (&v)[16]) {
  const lds_ptr<const lds_d2> q = (lds_ptr<const lds_d2>)p;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const lds_d2 t = q[i];
    v[2 * i] = t.x;
    v[2 * i + 1] = t.y;
  }
}

template <class MP>
__device__ void sy_tridiag64(MP A, int E, int lda, ldsd dg, ldsd od, ldsd bt, ldsd buf) {
  const int tid = threadIdx.x;
  // the wave index is uniform in the wave: in a scalar register, the
  // branches on it are scalar branches, not exec-mask updates
  const int q = __builtin_amdgcn_readfirstlane(tid >> 6), c = tid & 63;
  ldsd part = buf + 128;         // 4 x 64: partial A v of each wave
  ldsd wb = buf + 384 + 64 * q;  // 64 per wave (wave-private): w
  ldsd last = buf + 576;         // 2 x 64: rows E-2 and E-1 at the end
  ldsd part2 = buf + 704;        // 4 x 64: partial v^T X of each wave
  double a[16], x[16];
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) x[ii] = (16 * q + ii == c) ? 1.0 : 0.0;
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int r = 16 * q + ii;
    const double t = A[r * lda + c];  // r, c < 64 <= lda: in bounds
    a[ii] = ((r < E) & (c < E)) ? t : 0.0;  // no && here: a branch would serialise the loads
  }
  __syncthreads();  // A (LDS) now only receives reflector rows
  bool done = false;
  for (int jb = 0; jb < 4 && !done; ++jb) {
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = 16 * jb + jj;
      if (j + 2 >= E) {  // uniform
        done = true;
        break;
      }
      // the published row is double-buffered: a wave that skips the second
      // barrier of a step may publish the next row while others still read
      ldsd colb = buf + 64 * (jj & 1);
      if (q == jb) colb[c] = a[jj];  // row j = column j
      __syncthreads();
      const double col = colb[c];
      const double x0 = colb[j + 1];
      const double dj = colb[j];
      const double t = (c > j + 1) ? col : 0.0;
      const double xs2 = sum64(t * t);
      if (xs2 <= 1e-300 + 1e-32 * (xs2 + x0 * x0)) {  // already reduced (uniform)
        if (tid == 0) {
          bt[j] = 0.0;
          od[j] = x0;
          dg[j] = dj;
        }
        continue;
      }
      // sqrt and division from the hardware estimates with Newton steps: on
      // the critical path of every step
      const double s2 = xs2 + x0 * x0;
      const double alpha = s2 * rsq_acc(s2);
      const double sg = x0 >= 0.0 ? 1.0 : -1.0;
      const double v0 = x0 + sg * alpha;
      const double beta = 2.0 * rcp_acc(xs2 + v0 * v0);
      const double vc = (c == j + 1) ? v0 : t;
      // v on the own rows (zero on rows <= j): waves below jb hold no active row
      double vi[16];
      double pp = 0.0, px = 0.0;
      if (q >= jb) {
        lds_load16(colb + 16 * q, vi);
        if (q == jb) {
#pragma unroll
          for (int ii = 0; ii <= jj; ++ii) vi[ii] = 0.0;
          if (jj < 15) vi[(jj + 1) & 15] = v0;
        } else if (jj == 15 && q == jb + 1) {
          vi[0] = v0;
        }
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
        for (int ii = 0; ii < 16; ii += 4) {
          s0 = fma(a[ii], vi[ii], s0);
          s1 = fma(a[ii + 1], vi[ii + 1], s1);
          s2 = fma(a[ii + 2], vi[ii + 2], s2);
          s3 = fma(a[ii + 3], vi[ii + 3], s3);
        }
        pp = (s0 + s1) + (s2 + s3);
        double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
#pragma unroll
        for (int ii = 0; ii < 16; ii += 4) {
          u0 = fma(x[ii], vi[ii], u0);
          u1 = fma(x[ii + 1], vi[ii + 1], u1);
          u2 = fma(x[ii + 2], vi[ii + 2], u2);
          u3 = fma(x[ii + 3], vi[ii + 3], u3);
        }
        px = (u0 + u1) + (u2 + u3);
      }
      part[q * 64 + c] = pp;
      part2[q * 64 + c] = px;
      if (tid == 0) {
        dg[j] = dj;
        od[j] = -sg * alpha;
        bt[j] = beta;
      }
      __syncthreads();
      if (q >= jb) {
        const double p =
            beta * ((part[c] + part[64 + c]) + (part[128 + c] + part[192 + c]));
        const double K = 0.5 * beta * sum64(p * vc);
        const double w = p - K * vc;
        wb[c] = w;
        wave_lds_sync();
        double wi[16];
        lds_load16(wb + 16 * q, wi);
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) a[ii] = fma(-vi[ii], w, fma(-wi[ii], vc, a[ii]));
        // X <- H_j X = X - beta v (v^T X)
        const double bs =
            beta * ((part2[c] + part2[64 + c]) + (part2[128 + c] + part2[192 + c]));
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) x[ii] = fma(-bs, vi[ii], x[ii]);
        wave_lds_sync();  // wb is rewritten next step
      }
    }
  }
  // trailing 2 x 2 block (rows E-2, E-1)
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int r = 16 * q + ii;
    if (r >= E - 2 && r < E) last[(r - (E - 2)) * 64 + c] = a[ii];
  }
  __syncthreads();
  if (tid == 0) {
    if (E >= 2) {
      dg[E - 2] = last[E - 2];
      od[E - 2] = last[64 + E - 2];
      bt[E - 2] = 0.0;
    }
    dg[E - 1] = last[64 + E - 1];
    bt[E - 1] = 0.0;
  }
  // X = Q^T into A (A itself is no longer needed)
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) A[(16 * q + ii) * lda + c] = x[ii];
  __syncthreads();
}

// Tridiagonalisation for E <= 32 on the first wave alone; the other waves
// meet it only at the closing barrier.  Lane l holds column l & 31 of A (and
// of X), rows 16 (l >> 5) .. 16 (l >> 5) + 15, so the two halves of a column
// are one permlane32 swap apart: the column norm, A v, v^T X and p^T v are
// sums over the lane's own 16 rows plus one swap, with no lane reduction.
// The column, v and p reach every lane through LDS without a workgroup
// barrier, and v is formed in LDS (the published column with rows <= j + 1
// cleared by one store per lane, then v_{j+1}), so no lane masks its rows
// against the step index.  Same reflectors and outputs as sy_tridiag64 (dg,
// od, beta_j in bt[j], X = Q^T in A for rows and columns < E).
// buf: >= 160 doubles.
template <class MP>
__device__ void sy_tridiag32w(MP A, int E, int lda, ldsd dg, ldsd od, ldsd bt, ldsd buf) {
  if (threadIdx.x < 64) {
    const int l = threadIdx.x, c = l & 31, h = l >> 5;
    ldsd colA = buf;       // column j as it stands, 32
    ldsd colV = buf + 32;  // v of step j, 32
    ldsd pb = buf + 64;    // p, 32
    ldsd last = buf + 96;  // columns E-2 and E-1, 2 x 32
    double a[16], x[16];
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
      const int r = 16 * h + ii;
      const double t = A[r * lda + c];  // r, c < 32 < lda: in bounds
      a[ii] = ((r < E) & (c < E)) ? t : 0.0;
      x[ii] = (r == c) ? 1.0 : 0.0;
    }
    // LDS accesses of one wave complete in program order, and the fences
    // keep the compiler from moving them across the exchange points
    for (int j = 0; j + 2 < E; ++j) {
      if (c == j) {  // lanes j and j + 32: column j (= row j)
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) {
          colA[16 * h + ii] = a[ii];
          colV[16 * h + ii] = a[ii];
        }
      }
      if (l <= j + 1) colV[l] = 0.0;  // l <= j + 1 <= 30: rows that v leaves out
      wave_lds_sync();
      const double x0 = colA[j + 1], dj = colA[j];
      double m[16];
      lds_load16(colV + 16 * h, m);
      double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;
#pragma unroll
      for (int ii = 0; ii < 16; ii += 4) {
        n0 = fma(m[ii], m[ii], n0);
        n1 = fma(m[ii + 1], m[ii + 1], n1);
        n2 = fma(m[ii + 2], m[ii + 2], n2);
        n3 = fma(m[ii + 3], m[ii + 3], n3);
      }
      const double xs2 = sum_halves((n0 + n1) + (n2 + n3));  // same value in every lane
      if (xs2 <= 1e-300 + 1e-32 * (xs2 + x0 * x0)) {          // already reduced (uniform)
        if (l == 0) {
          bt[j] = 0.0;
          od[j] = x0;
          dg[j] = dj;
        }
        continue;
      }
      const double s2 = xs2 + x0 * x0;
      const double alpha = s2 * rsq_acc(s2);
      const double sg = x0 >= 0.0 ? 1.0 : -1.0;
      const double v0 = x0 + sg * alpha;
      const double beta = 2.0 * rcp_acc(xs2 + v0 * v0);
      if (l == 0) colV[j + 1] = v0;
      wave_lds_sync();
      double vi[16];
      lds_load16(colV + 16 * h, vi);
      const double vc = colV[c];
      double s0 = 0.0, s1 = 0.0, s2a = 0.0, s3 = 0.0, u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
#pragma unroll
      for (int ii = 0; ii < 16; ii += 4) {
        s0 = fma(a[ii], vi[ii], s0);
        s1 = fma(a[ii + 1], vi[ii + 1], s1);
        s2a = fma(a[ii + 2], vi[ii + 2], s2a);
        s3 = fma(a[ii + 3], vi[ii + 3], s3);
        u0 = fma(x[ii], vi[ii], u0);
        u1 = fma(x[ii + 1], vi[ii + 1], u1);
        u2 = fma(x[ii + 2], vi[ii + 2], u2);
        u3 = fma(x[ii + 3], vi[ii + 3], u3);
      }
      const double p = beta * sum_halves((s0 + s1) + (s2a + s3));   // (beta A v)_c
      const double bvx = beta * sum_halves((u0 + u1) + (u2 + u3));  // beta (v^T X)_c
      if (h == 0) pb[c] = p;
      if (l == 0) {
        dg[j] = dj;
        od[j] = -sg * alpha;
        bt[j] = beta;
      }
      wave_lds_sync();
      double pi[16];
      lds_load16(pb + 16 * h, pi);
      double k0 = 0.0, k1 = 0.0, k2 = 0.0, k3 = 0.0;
#pragma unroll
      for (int ii = 0; ii < 16; ii += 4) {
        k0 = fma(pi[ii], vi[ii], k0);
        k1 = fma(pi[ii + 1], vi[ii + 1], k1);
        k2 = fma(pi[ii + 2], vi[ii + 2], k2);
        k3 = fma(pi[ii + 3], vi[ii + 3], k3);
      }
      const double K = 0.5 * beta * sum_halves((k0 + k1) + (k2 + k3));
      // A - v w^T - w v^T with w = p - K v: entry (i, c) loses
      // v_i (p_c - 2 K v_c) + p_i v_c
      const double g = p - 2.0 * K * vc;
#pragma unroll
      for (int ii = 0; ii < 16; ++ii) {
        a[ii] = fma(-vi[ii], g, fma(-pi[ii], vc, a[ii]));
        x[ii] = fma(-bvx, vi[ii], x[ii]);
      }
    }
    // trailing 2 x 2 block: columns E-2 and E-1
    if (c == E - 2) {
#pragma unroll
      for (int ii = 0; ii < 16; ++ii) last[16 * h + ii] = a[ii];
    }
    if (c == E - 1) {
#pragma unroll
      for (int ii = 0; ii < 16; ++ii) last[32 + 16 * h + ii] = a[ii];
    }
    wave_lds_sync();
    if (l == 0) {
      if (E >= 2) {
        dg[E - 2] = last[E - 2];
        od[E - 2] = last[E - 1];
        bt[E - 2] = 0.0;
      }
      if (E >= 1) {
        dg[E - 1] = last[32 + E - 1];
        bt[E - 1] = 0.0;
      }
    }
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) A[(16 * h + ii) * lda + c] = x[ii];
  }
  __syncthreads();
}

// The same reduction for E <= 16, with four rows per lane: lane l holds
// column l & 15, rows 4 (l >> 4) .. 4 (l >> 4) + 3, so a column's four row
// groups are the four DPP rows at one position and every per-column sum is
// a sum over the own four rows plus sum_rows4.  buf: >= 96 doubles.
template <class MP>
__device__ void sy_tridiag16w(MP A, int E, int lda, ldsd dg, ldsd od, ldsd bt, ldsd buf) {
  if (threadIdx.x < 64) {
    const int l = threadIdx.x, c = l & 15, g = l >> 4;
    ldsd colA = buf;       // column j as it stands, 16
    ldsd colV = buf + 16;  // v of step j, 16
    ldsd pb = buf + 32;    // p, 16
    ldsd last = buf + 48;  // columns E-2 and E-1, 2 x 16
    double a[4], x[4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int r = 4 * g + ii;
      const double t = A[r * lda + c];  // r, c < 16 < lda: in bounds
      a[ii] = ((r < E) & (c < E)) ? t : 0.0;
      x[ii] = (r == c) ? 1.0 : 0.0;
    }
    for (int j = 0; j + 2 < E; ++j) {
      if (c == j) {  // the four lanes of column j (= row j)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          colA[4 * g + ii] = a[ii];
          colV[4 * g + ii] = a[ii];
        }
      }
      if (l <= j + 1) colV[l] = 0.0;  // l <= j + 1 <= 14: rows that v leaves out
      wave_lds_sync();
      const double x0 = colA[j + 1], dj = colA[j];
      double m[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) m[ii] = colV[4 * g + ii];
      const double xs2 = sum_rows4(fma(m[0], m[0], m[1] * m[1]) + fma(m[2], m[2], m[3] * m[3]));
      if (xs2 <= 1e-300 + 1e-32 * (xs2 + x0 * x0)) {  // already reduced (uniform)
        if (l == 0) {
          bt[j] = 0.0;
          od[j] = x0;
          dg[j] = dj;
        }
        continue;
      }
      const double s2 = xs2 + x0 * x0;
      const double alpha = s2 * rsq_acc(s2);
      const double sg = x0 >= 0.0 ? 1.0 : -1.0;
      const double v0 = x0 + sg * alpha;
      const double beta = 2.0 * rcp_acc(xs2 + v0 * v0);
      if (l == 0) colV[j + 1] = v0;
      wave_lds_sync();
      double vi[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) vi[ii] = colV[4 * g + ii];
      const double vc = colV[c];
      const double p =
          beta * sum_rows4(fma(a[0], vi[0], a[1] * vi[1]) + fma(a[2], vi[2], a[3] * vi[3]));
      const double bvx =
          beta * sum_rows4(fma(x[0], vi[0], x[1] * vi[1]) + fma(x[2], vi[2], x[3] * vi[3]));
      if (g == 0) pb[c] = p;
      if (l == 0) {
        dg[j] = dj;
        od[j] = -sg * alpha;
        bt[j] = beta;
      }
      wave_lds_sync();
      double pi[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) pi[ii] = pb[4 * g + ii];
      const double K = 0.5 * beta *
                       sum_rows4(fma(pi[0], vi[0], pi[1] * vi[1]) + fma(pi[2], vi[2], pi[3] * vi[3]));
      // A - v w^T - w v^T with w = p - K v (as in sy_tridiag32w)
      const double gg = p - 2.0 * K * vc;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        a[ii] = fma(-vi[ii], gg, fma(-pi[ii], vc, a[ii]));
        x[ii] = fma(-bvx, vi[ii], x[ii]);
      }
    }
    if (c == E - 2) {
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) last[4 * g + ii] = a[ii];
    }
    if (c == E - 1) {
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) last[16 + 4 * g + ii] = a[ii];
    }
    wave_lds_sync();
    if (l == 0) {
      if (E >= 2) {
        dg[E - 2] = last[E - 2];
        od[E - 2] = last[E - 1];
        bt[E - 2] = 0.0;
      }
      if (E >= 1) {
        dg[E - 1] = last[16 + E - 1];
        bt[E - 1] = 0.0;
      }
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) A[(4 * g + ii) * lda + c] = x[ii];
  }
  __syncthreads();
}

// Z <- Q Z for the r <= 64 columns of Z (E <= 64 rows) with X = Q^T in A
// (sy_tridiag64), as one product on the FP64 matrix cores: wave w forms the
// 16-row block w of U = X^T Z, one 16 x 16 block per 16 columns.  All
// threads; Z is read completely before it is overwritten.
typedef double syev_f64x4 __attribute__((ext_vector_type(4)));

template <int NBJ, class MP>
__device__ __forceinline__ void backtr_gemm64_n(MP X, int E, int lda, MP Z, int r) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
  syev_f64x4 acc[NBJ];
#pragma unroll
  for (int t = 0; t < NBJ; ++t) acc[t] = syev_f64x4{0.0, 0.0, 0.0, 0.0};
  // sixteen rows of Z per pass, four products each, with no branch inside
  // (operands loaded first, accumulators stay in place)
  for (int k16 = 0; k16 < E; k16 += 16) {
    double a[4], bz[4][NBJ];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int c = k16 + 4 * u + lk;
      const bool cin = c < E;
      const int cc = cin ? c : 0;
      const double av = X[cc * lda + 16 * w + lr];  // X^T(i, c), i = 16w + lr < 64 <= lda
      a[u] = cin ? av : 0.0;
#pragma unroll
      for (int t = 0; t < NBJ; ++t) {
        const double bv = Z[cc * lda + 16 * t + lr];  // column < 64 <= lda
        bz[u][t] = cin ? bv : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < NBJ; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], bz[u][t], acc[t], 0, 0, 0);
  }
  __syncthreads();  // every wave has read Z
#pragma unroll
  for (int t = 0; t < NBJ; ++t) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * w + 4 * e + lk, b = 16 * t + lr;
      if (i < E && b < r) Z[i * lda + b] = acc[t][e];
    }
  }
  __syncthreads();
}

template <class MP>
__device__ void backtr_gemm64(MP X, int E, int lda, MP Z, int r) {
  const int nbj = (r + 15) >> 4;  // <= 4, uniform
  if (nbj <= 1)
    backtr_gemm64_n<1>(X, E, lda, Z, r);
  else if (nbj == 2)
    backtr_gemm64_n<2>(X, E, lda, Z, r);
  else if (nbj == 3)
    backtr_gemm64_n<3>(X, E, lda, Z, r);
  else
    backtr_gemm64_n<4>(X, E, lda, Z, r);
}


// Orthonormalisation of the r <= 32 kept eigenvectors of T (columns of Z,
// E <= 64 rows) when they are already orthonormal to first order, then
// Z <- Q Z (backtr_gemm64).  Vectors from the twisted factorisation are
// orthogonal to about u ||T|| / gap; with C = Z^T Z and D = C - I, one
// Newton-Schulz step Z <- Z (3I - C) / 2 leaves an error of order ||D||^2,
// so for max |D| <= 1e-8 it restores orthonormality to rounding level at the
// cost of two small products on the matrix cores.  Otherwise (clustered
// eigenvalues) the routine returns false with Z untouched and the caller
// takes the Gram-Schmidt path.  All threads; cs: >= 32 * 32 + 8 doubles.
template <class MP>
__device__ bool polish_backtr64(MP A, int E, int lda, MP Z, int r, ldsd cs) {
  constexpr int LC = 32;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  ldsd S = cs;               // C, then (3I - C) / 2, r x r (stride LC)
  ldsd dev = cs + 32 * LC;  // per-wave max |C - I|
  const int nb = (r + 15) >> 4;  // <= 2
  double dmax = 0.0;
  if (w < nb * nb) {  // <= 4 blocks: one per wave
    const int blk = w;
    const int bi = blk / nb, bj = blk - bi * nb;
    syev_f64x4 acc = syev_f64x4{0.0, 0.0, 0.0, 0.0};
    for (int k16 = 0; k16 < E; k16 += 16) {  // operands first, no branch among the products
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = k16 + 4 * u + lk;
        const bool cin = c < E;
        const int cc = cin ? c : 0;
        const double a = Z[cc * lda + 16 * bi + lr], bz = Z[cc * lda + 16 * bj + lr];
        av[u] = cin ? a : 0.0;
        bv[u] = cin ? bz : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * bi + 4 * e + lk, j = 16 * bj + lr;
      if (i < r && j < r) {
        const double d = acc[e] - (i == j ? 1.0 : 0.0);
        dmax = fmax(dmax, fabs(d));
        if (!(d == d)) dmax = 1.0;  // NaN
        S[i * LC + j] = (i == j ? 1.0 : 0.0) - 0.5 * d;
      }
    }
  }
  dmax = max64(dmax);
  if (l == 0) dev[w] = dmax;
  __syncthreads();
  const double dm = fmax(fmax(dev[0], dev[1]), fmax(dev[2], dev[3]));
  if (!(dm <= 1e-8)) return false;  // uniform; Z untouched
  // Z' = Z S: 16 x 16 blocks (row block rb < 4, column block cb < nb) over the waves
  syev_f64x4 zo[2];
  const int nrb = (E + 15) >> 4;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    zo[t] = syev_f64x4{0.0, 0.0, 0.0, 0.0};
    const int blk = w + 4 * t;
    if (blk >= nrb * nb) continue;  // uniform
    const int rb = blk / nb, cb = blk - rb * nb;
    const int row = 16 * rb + lr;
    const bool rin = row < E;
    const int rr = rin ? row : 0;
    for (int k16 = 0; k16 < r; k16 += 16) {  // operands first, no branch among the products
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k16 + 4 * u + lk;
        const bool kin = kk < r;
        const int kc = kin ? kk : 0;
        const double a = Z[rr * lda + kc];
        const double b = S[kc * LC + 16 * cb + lr];
        av[u] = (rin & kin) ? a : 0.0;
        bv[u] = kin ? b : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        zo[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], zo[t], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read Z
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int blk = w + 4 * t;
    if (blk >= nrb * nb) continue;
    const int rb = blk / nb, cb = blk - rb * nb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * rb + 4 * e + lk, j = 16 * cb + lr;
      if (i < E && j < r) Z[i * lda + j] = zo[t][e];
    }
  }
  __syncthreads();
  backtr_gemm64(A, E, lda, Z, r);
  return true;
}

// The same for 32 < r <= 64 kept eigenvectors (columns of Z,
// E <= 64 rows) when they are already orthonormal to first order, with the
// back-transformation.  Vectors from the twisted factorisation are
// orthogonal to about u ||T|| / gap (as above).  S no longer fits the
// scratch, so C is formed first (up to four 16 x 16 blocks per wave, kept in registers); when
// the test passes, Z <- Q Z (backtr_gemm64), which frees A, S = (3I - C) / 2
// goes into A and Z <- Z S (Q Z S = Q (Z S)).  Otherwise (clustered
// eigenvalues) the routine returns false with Z untouched and the caller
// takes the Gram-Schmidt path.  All threads; cs: >= 8 doubles.
template <class MP>
__device__ bool polish_backtr64_wide(MP A, int E, int lda, MP Z, int r, ldsd cs) {
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, lr = l & 15, lk = l >> 4;
  ldsd dev = cs;  // per-wave max |C - I|
  const int nb = (r + 15) >> 4;  // <= 4
  double dmax = 0.0;
  syev_f64x4 cacc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    cacc[t] = syev_f64x4{0.0, 0.0, 0.0, 0.0};
    const int blk = w + 4 * t;
    if (blk >= nb * nb) continue;  // wave-uniform
    const int bi = blk / nb, bj = blk - bi * nb;
    for (int k16 = 0; k16 < E; k16 += 16) {  // operands first, no branch among the products
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = k16 + 4 * u + lk;
        const bool cin = c < E;
        const int cc = cin ? c : 0;
        const double a = Z[cc * lda + 16 * bi + lr], bz = Z[cc * lda + 16 * bj + lr];
        av[u] = cin ? a : 0.0;
        bv[u] = cin ? bz : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        cacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], cacc[t], 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * bi + 4 * e + lk, j = 16 * bj + lr;
      if (i < r && j < r) {
        const double d = cacc[t][e] - (i == j ? 1.0 : 0.0);
        dmax = fmax(dmax, fabs(d));
        if (!(d == d)) dmax = 1.0;  // NaN
      }
    }
  }
  dmax = max64(dmax);
  if (l == 0) dev[w] = dmax;
  __syncthreads();
  const double dm = fmax(fmax(dev[0], dev[1]), fmax(dev[2], dev[3]));
  if (!(dm <= 1e-8)) return false;  // uniform; Z untouched
  backtr_gemm64(A, E, lda, Z, r);   // Z <- Q Z; A is free from here
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int blk = w + 4 * t;
    if (blk >= nb * nb) continue;
    const int bi = blk / nb, bj = blk - bi * nb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * bi + 4 * e + lk, j = 16 * bj + lr;
      if (i < r && j < r) {
        const double d = cacc[t][e] - (i == j ? 1.0 : 0.0);
        A[i * lda + j] = (i == j ? 1.0 : 0.0) - 0.5 * d;
      }
    }
  }
  __syncthreads();
  // Z' = Z S: 16 x 16 blocks (row block rb < nrb, column block cb < nb)
  syev_f64x4 zo[4];
  const int nrb = (E + 15) >> 4;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    zo[t] = syev_f64x4{0.0, 0.0, 0.0, 0.0};
    const int blk = w + 4 * t;
    if (blk >= nrb * nb) continue;  // wave-uniform
    const int rb = blk / nb, cb = blk - rb * nb;
    const int row = 16 * rb + lr;
    const bool rin = row < E;
    const int rr = rin ? row : 0;
    for (int k16 = 0; k16 < r; k16 += 16) {
      double av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = k16 + 4 * u + lk;
        const bool kin = kk < r;
        const int kc = kin ? kk : 0;
        const double a = Z[rr * lda + kc];
        const double b = A[kc * lda + 16 * cb + lr];
        av[u] = (rin & kin) ? a : 0.0;
        bv[u] = kin ? b : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        zo[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], zo[t], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave has read Z
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int blk = w + 4 * t;
    if (blk >= nrb * nb) continue;
    const int rb = blk / nb, cb = blk - rb * nb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = 16 * rb + 4 * e + lk, j = 16 * cb + lr;
      if (i < E && j < r) Z[i * lda + j] = zo[t][e];
    }
  }
  __syncthreads();
  return true;
}

// Modified Gram-Schmidt of the r kept eigenvectors of T (columns 0..r-1 of
// Z, E <= 64 rows, r <= 64) in registers, followed by Z <- Q Z with the
// accumulated Q^T of sy_tridiag64 in A.  Column b lives in wave b / 16, in the
// lanes at position b % 16 of the four DPP rows, row q holding entries
// 16q..16q+15; a dot product is a per-lane sum plus two lane swaps.  Step j
// publishes column j (as it stands, unnormalised) and 1 / ||z_j||^2 in a
// double-buffered LDS slot (pub: 2 x 72 doubles) and every later column
// removes its projection on it; one barrier per step.  The columns are
// normalised at the end.  A column that keeps less than a quarter of its
// norm (a repeated eigenvalue: the twisted factorisation returned the same
// vector twice) makes the routine return false with Z untouched, and the
// caller takes mgs_cols, whose inverse iteration replaces such columns.
template <class MP>
__device__ bool mgs_backtr64(MP A, int E, int lda, MP Z, int ldz, int r, ldsd pub, ldsi flag) {
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, q = l >> 4;
  const int b = 16 * w + (l & 15);
  const bool own = b < r;
  const int bl = own ? b : 0;
  double z[16];
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int i = 16 * q + ii;
    const double t = Z[i * ldz + bl];  // i < 64 rows, bl < 64 <= ldz: in bounds
    z[ii] = (i < E) ? t : 0.0;         // other lanes' values are never stored
  }
  if (tid == 0) flag[0] = 0;
  double nz = 1.0;  // squared norm of the own column when it was published
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    ldsd slot = pub + 72 * (j & 1);
    if (w == (j >> 4)) {
      const bool pubr = (l & 15) == (j & 15);
      if (pubr) {
#pragma unroll
        for (int ii = 0; ii < 16; ++ii) slot[16 * q + ii] = z[ii];
      }
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int ii = 0; ii < 16; ii += 4) {
        s0 = fma(z[ii], z[ii], s0);
        s1 = fma(z[ii + 1], z[ii + 1], s1);
        s2 = fma(z[ii + 2], z[ii + 2], s2);
        s3 = fma(z[ii + 3], z[ii + 3], s3);
      }
      const double sn = sum_rows4((s0 + s1) + (s2 + s3));
      if (pubr) {
        nz = sn;
        if (l == (j & 15)) {
          slot[64] = sn > 0.0 ? rcp_acc(sn) : 0.0;
          if (j > 0 && !(sn >= 0.25)) flag[0] = 1;
        }
      }
    }
    __syncthreads();
    double pj[16];
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) pj[ii] = slot[16 * q + ii];
    const double is = slot[64];
    double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
    for (int ii = 0; ii < 16; ii += 4) {
      p0 = fma(pj[ii], z[ii], p0);
      p1 = fma(pj[ii + 1], z[ii + 1], p1);
      p2 = fma(pj[ii + 2], z[ii + 2], p2);
      p3 = fma(pj[ii + 3], z[ii + 3], p3);
    }
    // no branch around the update: the compiler would sink the load of is
    // into it and serialise a second LDS round trip
    const double d = (own && b > j) ? sum_rows4((p0 + p1) + (p2 + p3)) * is : 0.0;
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) z[ii] = fma(-d, pj[ii], z[ii]);
  }
  __syncthreads();
  if (flag[0]) return false;  // uniform; Z was not written
  {
    const double inv = nz > 0.0 ? rsq_acc(nz) : 0.0;
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) z[ii] *= inv;
  }
  if (16 * w < r) {
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) {
      const int i = 16 * q + ii;
      if (own && i < E) Z[i * ldz + b] = z[ii];
    }
  }
  __syncthreads();
  backtr_gemm64(A, E, lda, Z, r);
  return true;
}

// Sturm counts (number of eigenvalues below x[t]) for NC shifts at once, on
// T scaled to ||T|| ~ 1 (diagonal dn, squared off-diagonal e2n).  Three-term
// recurrence of the leading principal minors
//   p_i = (a_i - x) p_{i-1} - b_{i-1}^2 p_{i-2},  p_0 = 1,
// counting sign changes.  An exact zero p_i needs no special case: then
// p_{i+1} = -b_i^2 p_{i-1} has the sign opposite to p_{i-1}, so the pair of
// steps contributes one change whatever sign the zero is given.  Division-
// free: one FMA on the dependent path per step.  The pair (p_i, p_{i-1}) is
// rescaled by a power of two every 8 steps; with |a - x| <= 3 and b^2 in
// [1e-60, 1] it grows at most 4^8-fold and shrinks at most 1e-240-fold in
// between, within the normal double range.
__device__ __forceinline__ int sign_change(double a, double b) {
  return (int)(((unsigned int)(__double2hiint(a) ^ __double2hiint(b))) >> 31);
}

template <int NC>
__device__ __forceinline__ void sturm_counts(lds_ptr<const double> dn, lds_ptr<const double> e2n, int E,
                                             const double* x, int* c) {
  double pm[NC], pc[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    pm[t] = 1.0;
    pc[t] = dn[0] - x[t];
    c[t] = sign_change(pc[t], 1.0);
  }
  auto step = [&](double a, double b2) {
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const double pn = fma(a - x[t], pc[t], -b2 * pm[t]);
      c[t] += sign_change(pn, pc[t]);
      pm[t] = pc[t];
      pc[t] = pn;
    }
  };
  int i = 1;
  for (; i + 7 < E; i += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = dn[i + u];
      bv[u] = e2n[i - 1 + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) step(av[u], bv[u]);
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pc[t]), fabs(pm[t])));
      pc[t] = ldexp(pc[t], -ex);
      pm[t] = ldexp(pm[t], -ex);
    }
  }
  for (; i < E; ++i) step(dn[i], e2n[i - 1]);
}

// Multisection over NC chains per lane: a 16-lane group brackets the
// eigenvalues k = g, g + NT/16, ... and shrinks each bracket 17x per pass.
template <int NT, int NC>
__device__ void multisect(lds_ptr<const double> dn, lds_ptr<const double> e2n, int E, double lo,
                          double hi, double width_stop, double scale, ldsd lam) {
  const int tid = threadIdx.x;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG16 = NT / 16;
  int nk = 0;
  for (int k = g16; k < E; k += NG16) ++nk;
  if (nk == 0) return;
  const int gshift = (tid & 48);  // first lane of the 16-group within the wave
  const double frac = (double)(l16 + 1) * (1.0 / 17.0);
  double l[NC], u[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    l[t] = lo;
    u[t] = hi;
  }
  for (int it = 0; it < 40; ++it) {
    // all brackets shrink by the same factor, so one test serves every chain
    if (!((u[0] - l[0]) > width_stop)) break;
    double x[NC];
    int c[NC];
#pragma unroll
    for (int t = 0; t < NC; ++t) x[t] = l[t] + (u[t] - l[t]) * frac;
    sturm_counts<NC>(dn, e2n, E, x, c);
#pragma unroll
    for (int t = 0; t < NC; ++t) {
      const int k = g16 + t * NG16;
      const unsigned long long b = __ballot(c[t] > k);
      const unsigned int gb = (unsigned int)((b >> gshift) & 0xFFFFull);
      const int first = gb ? __builtin_ctz(gb) : 16;
      const double w = (u[t] - l[t]) * (1.0 / 17.0);
      const double nl = (first == 0) ? l[t] : l[t] + w * (double)first;
      const double nu = (first == 16) ? u[t] : l[t] + w * (double)(first + 1);
      l[t] = nl;
      u[t] = nu;
    }
  }
#pragma unroll
  for (int t = 0; t < NC; ++t)
    if (t < nk && l16 == 0) lam[g16 + t * NG16] = 0.5 * (l[t] + u[t]) * scale;
}

// Sturm counts on T padded to NE rows: beyond E the diagonal is 4 and the
// squared off-diagonal 0 (tridiag_eigvals writes the padding), steps that
// keep the sign of the minor and so add no change.  Same recurrence and
// rescaling as sturm_counts; the signs of p_1 .. p_NE are shifted into a bit
// mask, one alignbit per step, and the changes are counted once at the end:
// with s_0 = 0 (p_0 = 1) and bit k of M holding s_{NE-k}, the changes are
// the set bits of M xor (M >> 1).
__device__ __forceinline__ unsigned int shift_sign(unsigned int m, double p) {
  return __builtin_amdgcn_alignbit(m, (unsigned int)__double2hiint(p), 31);
}

template <int NE>
__device__ __forceinline__ int sign_mask_changes(unsigned int mh, unsigned int ml) {
  if constexpr (NE <= 32) {
    return __popc(mh ^ (mh >> 1));
  } else {
    // mh holds s_1 .. s_32, ml the remaining NE - 32 signs
    const unsigned long long m = ((unsigned long long)mh << (NE - 32)) | ml;
    return __popcll(m ^ (m >> 1));
  }
}

// registers: av[i] = a_i, bv[i] = b_{i-1}^2 (bv[0] unused), NE <= 32
template <int NE>
__device__ __forceinline__ int sturm_count_reg(const double* av, const double* bv, double x) {
  static_assert(NE <= 32, "one 32-bit sign mask");
  double pm = 1.0, pc = av[0] - x;
  unsigned int mh = shift_sign(0u, pc);
#pragma unroll
  for (int i = 1; i < NE; ++i) {
    const double pn = fma(av[i] - x, pc, -bv[i] * pm);
    mh = shift_sign(mh, pn);
    pm = pc;
    pc = pn;
    if ((i & 7) == 0) {
      const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pc), fabs(pm)));
      pc = ldexp(pc, -ex);
      pm = ldexp(pm, -ex);
    }
  }
  return sign_mask_changes<NE>(mh, 0u);
}

// LDS operands, NE = 48 or 64: dn[0..NE) and e2n[0..NE-1) padded; loads
// in blocks of 8
template <int NE>
__device__ __forceinline__ int sturm_count_lds(lds_ptr<const double> dn,
                                               lds_ptr<const double> e2n, double x) {
  static_assert(NE > 32 && NE <= 64, "two sign masks");
  double pm = 1.0, pc = dn[0] - x;
  unsigned int mh = shift_sign(0u, pc), ml = 0u;
#pragma unroll
  for (int i0 = 1; i0 < NE; i0 += 8) {
    double av[8], bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      av[u] = (i0 + u < NE) ? dn[i0 + u] : 0.0;
      bv[u] = (i0 + u < NE) ? e2n[i0 - 1 + u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u;
      if (i < NE) {
        const double pn = fma(av[u] - x, pc, -bv[u] * pm);
        if (i < 32)
          mh = shift_sign(mh, pn);
        else
          ml = shift_sign(ml, pn);
        pm = pc;
        pc = pn;
        if ((i & 7) == 0) {
          const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pc), fabs(pm)));
          pc = ldexp(pc, -ex);
          pm = ldexp(pm, -ex);
        }
      }
    }
  }
  return sign_mask_changes<NE>(mh, ml);
}

// Multisection for the K largest eigenvalues (K <= 256 / G) with a group of
// G lanes per eigenvalue: group g brackets eigenvalue E-1-g (ascending
// index) and narrows its bracket (G+1)x per pass with one Sturm count per
// lane.  All brackets start equal and shrink by the same factor, so the pass
// count is fixed up front.  T is padded to NE rows; for NE <= 32 it is read
// from LDS once and every pass runs on registers, for NE = 48 or 64 from LDS
// in blocks of 8.
template <int NT, int G, int NE>
__device__ void multisect_top_pad(lds_ptr<const double> dn, lds_ptr<const double> e2n, int E,
                                  int K, double lo, double hi, double width_stop, double scale,
                                  ldsd lam) {
  static_assert(NT == 256 && (G == 4 || G == 8 || G == 16), "lane groups of a 256-thread block");
  const int tid = threadIdx.x;
  const int grp = tid / G, lg = tid & (G - 1);
  const int k = E - 1 - grp;
  const int gshift = (tid & 63) & ~(G - 1);
  const double frac = (double)(lg + 1) * (1.0 / (double)(G + 1));
  const int passes = (int)ceil(log((hi - lo) / width_stop) / log((double)(G + 1)));
  double av[NE <= 32 ? NE : 1], bv[NE <= 32 ? NE : 1];
  if constexpr (NE <= 32) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      av[i] = dn[i];
      bv[i] = (i >= 1) ? e2n[i - 1] : 0.0;
    }
  }
  double l = lo, u = hi;
  for (int it = 0; it < passes; ++it) {
    const double x = l + (u - l) * frac;
    int c;
    if constexpr (NE <= 32)
      c = sturm_count_reg<NE>(av, bv, x);
    else
      c = sturm_count_lds<NE>(dn, e2n, x);
    const unsigned long long bal = __ballot(c > k);
    const unsigned int gb = (unsigned int)((bal >> gshift) & ((1ull << G) - 1));
    const int first = gb ? __builtin_ctz(gb) : G;
    const double w = (u - l) * (1.0 / (double)(G + 1));
    const double nl = (first == 0) ? l : l + w * (double)first;
    const double nu = (first == G) ? u : l + w * (double)(first + 1);
    l = nl;
    u = nu;
  }
  if (lg == 0 && grp < K && k >= 0) lam[k] = 0.5 * (l + u) * scale;
}

template <int NT, int G>
__device__ void multisect_top_any(lds_ptr<const double> dn, lds_ptr<const double> e2n, int E,
                                  int K, double lo, double hi, double width_stop, double scale,
                                  ldsd lam) {
  if (E <= 8)
    multisect_top_pad<NT, G, 8>(dn, e2n, E, K, lo, hi, width_stop, scale, lam);
  else if (E <= 16)
    multisect_top_pad<NT, G, 16>(dn, e2n, E, K, lo, hi, width_stop, scale, lam);
  else if (E <= 24)
    multisect_top_pad<NT, G, 24>(dn, e2n, E, K, lo, hi, width_stop, scale, lam);
  else if (E <= 32)
    multisect_top_pad<NT, G, 32>(dn, e2n, E, K, lo, hi, width_stop, scale, lam);
  else if (E <= 48)
    multisect_top_pad<NT, G, 48>(dn, e2n, E, K, lo, hi, width_stop, scale, lam);
  else
    multisect_top_pad<NT, G, 64>(dn, e2n, E, K, lo, hi, width_stop, scale, lam);
}

// All eigenvalues of T in ascending order into lam[0..E), to an absolute
// accuracy of about 1e-15 ||T||.  e2, dn: >= E doubles of scratch each.
template <int NT>
__device__ void tridiag_eigvals(lds_ptr<const double> dg, lds_ptr<const double> od, int E, ldsd lam,
                                ldsd e2, ldsd dn, double nrm, int K) {
  // nrm: the Gershgorin bound of T (tridiag_gersh); for E <= 64 only the K
  // largest eigenvalues are computed (lam[E-K..E)), otherwise all
  const int tid = threadIdx.x;
  if (!(nrm > 0.0)) {
    for (int i = tid; i < E; i += NT) lam[i] = 0.0;
    __syncthreads();
    return;
  }
  const double sc = 1.0 / nrm;
  for (int i = tid; i < E; i += NT) {
    dn[i] = dg[i] * sc;
    if (i + 1 < E) {
      const double b = od[i] * sc;
      e2[i] = fmax(b * b, 1e-60);
    }
  }
  // padding to 64 rows for the fixed-length counts (multisect_top_pad):
  // diagonal 4, off-diagonal 0 (dn, e2: >= 64 doubles)
  if (E <= 64) {
    for (int i = E + tid; i < 64; i += NT) dn[i] = 4.0;
    for (int i = E - 1 + tid; i < 64; i += NT)
      if (i >= 0) e2[i] = 0.0;
  }
  __syncthreads();
  // scaled Gershgorin interval lies inside [-1, 1]; widen by the stop width
  const double ws = 1e-15;
  constexpr int NG16 = NT / 16;
  const int nkmax = (E + NG16 - 1) / NG16;
  // (5x per pass: stop at 2e-16, below the 17x scheme's last width, since the
  // eigenvector error of the twisted factorisation follows the eigenvalue's)
  if (NT == 256 && E <= 64) {
    // only the K largest (ascending slots E-K..E-1 of lam); finer groups
    // when fewer are wanted, fewer passes
    if (K <= 16)
      multisect_top_any<NT, 16>(dn, e2, E, K, -1.0 - ws, 1.0 + ws, 2e-16, nrm, lam);
    else if (K <= 32)
      multisect_top_any<NT, 8>(dn, e2, E, K, -1.0 - ws, 1.0 + ws, 2e-16, nrm, lam);
    else
      multisect_top_any<NT, 4>(dn, e2, E, K, -1.0 - ws, 1.0 + ws, 2e-16, nrm, lam);
  } else if (nkmax <= 1)
    multisect<NT, 1>(dn, e2, E, -1.0 - ws, 1.0 + ws, ws, nrm, lam);
  else if (nkmax <= 2)
    multisect<NT, 2>(dn, e2, E, -1.0 - ws, 1.0 + ws, ws, nrm, lam);
  else if (nkmax <= 4)
    multisect<NT, 4>(dn, e2, E, -1.0 - ws, 1.0 + ws, ws, nrm, lam);
  else
    multisect<NT, 8>(dn, e2, E, -1.0 - ws, 1.0 + ws, ws, nrm, lam);
  __syncthreads();
}

// Eigenvector of T for eigenvalue lam by a twisted factorisation; written
// (normalised) to z[i*ldz] for i < E.  One lane per vector.
template <class MP>
__device__ inline void tridiag_vec(lds_ptr<const double> dg, lds_ptr<const double> od, int E,
                                   double lam, MP z, int ldz, double tiny) {
  if (E == 1) {
    z[0] = 1.0;
    return;
  }
  // top-down: T - lam I = L D+ L^T ; l_i stored in z[i]
  double dp = dg[0] - lam;
  if (fabs(dp) < tiny) dp = tiny;
  double gam_best = 1e308;
  int rbest = 0;
  // keep D+ values to form gamma: recompute on the bottom-up sweep instead
  for (int i = 0; i + 1 < E; ++i) {
    const double li = od[i] * rcp_acc(dp);
    z[i * ldz] = li;
    dp = (dg[i + 1] - lam) - li * od[i];
    if (fabs(dp) < tiny) dp = tiny;
  }
  // bottom-up: T - lam I = U D- U^T ; gamma_r = D+_r + D-_r - (a_r - lam)
  // (D+_r recomputed from the stored l: D+_{i+1} = a_{i+1} - lam - l_i b_i)
  double dm = dg[E - 1] - lam;
  if (fabs(dm) < tiny) dm = tiny;
  {
    // D+_{E-1}
    const double dpl = (dg[E - 1] - lam) - z[(E - 2) * ldz] * od[E - 2];
    const double g = dpl + dm - (dg[E - 1] - lam);
    gam_best = fabs(g);
    rbest = E - 1;
  }
  for (int i = E - 1; i >= 1; --i) {
    const double ui = od[i - 1] * rcp_acc(dm);
    dm = (dg[i - 1] - lam) - ui * od[i - 1];
    if (fabs(dm) < tiny) dm = tiny;
    const double dpl = (i - 1 == 0) ? (dg[0] - lam)
                                    : (dg[i - 1] - lam) - z[(i - 2) * ldz] * od[i - 2];
    const double g = dpl + dm - (dg[i - 1] - lam);
    if (fabs(g) < gam_best) {
      gam_best = fabs(g);
      rbest = i - 1;
    }
  }
  const int r = rbest;
  // u_i for i > r (recomputed bottom-up), stored in z[i] (the l there is no longer needed)
  dm = dg[E - 1] - lam;
  if (fabs(dm) < tiny) dm = tiny;
  for (int i = E - 1; i > r; --i) {
    const double ui = od[i - 1] * rcp_acc(dm);
    z[i * ldz] = ui;
    dm = (dg[i - 1] - lam) - ui * od[i - 1];
    if (fabs(dm) < tiny) dm = tiny;
  }
  // z_r = 1; upward z_i = -l_i z_{i+1} (i < r); downward z_{i+1} = -u_{i+1} z_i (i >= r)
  double nrm2 = 1.0;
  double zc = 1.0;
  for (int i = r - 1; i >= 0; --i) {
    zc = -z[i * ldz] * zc;
    z[i * ldz] = zc;
    nrm2 = fma(zc, zc, nrm2);
  }
  zc = 1.0;
  for (int i = r; i + 1 < E; ++i) {
    zc = -z[(i + 1) * ldz] * zc;
    z[(i + 1) * ldz] = zc;
    nrm2 = fma(zc, zc, nrm2);
  }
  z[r * ldz] = 1.0;
  const double inv = 1.0 / sqrt(nrm2);
  for (int i = 0; i < E; ++i) z[i * ldz] *= inv;
}

// The same twisted factorisation with two lanes per vector, for r <= 32
// vectors (wave 0): lane b sweeps top-down (T - lam I = L D+ L^T, l_i into
// column b of Z) while lane b + 32 sweeps bottom-up (U D- U^T, u_i into
// column b + 32, free since r <= 32); both run one instruction stream with
// mirrored indices.  The twist index minimises
//   |gamma_i| = |(a_i - lam) - l_{i-1} b_{i-1} - u_{i+1} b_i|
// (ties to the larger index), each lane scanning half of i; then lane b
// builds the vector upward from it (z_i = -l_i z_{i+1}) and lane b + 32
// downward (z_i = -u_i z_{i-1}), both into column b, which is normalised.
template <class MP>
__device__ void tridiag_vec_pair(lds_ptr<const double> dg, lds_ptr<const double> od, int E,
                                 lds_ptr<const double> lam, MP Z, int ldz, int r, double tiny) {
  const int l = threadIdx.x & 63;
  const int b = l & 31, hb = l >> 5;
  const bool act = b < r;
  const double lm = lam[act ? b : 0];
  MP zc = Z + b;
  MP own = Z + b + 32 * hb;  // where this lane's sweep stores l_i or u_i
  if (E == 1) {
    if (act && hb == 0) zc[0] = 1.0;
    wave_lds_sync();
    return;
  }
  // The two halves mirror each other: every row index below is linear in
  // the step with slope dir (+1 top-down, -1 bottom-up), so the lanes
  // compute their indices without branches.  Lanes without a vector (b >= r)
  // run the same steps on lam[0] and write only columns that no later step
  // reads.
  const int dir = hb ? -1 : 1;
  // sweeps: step t handles row is = t (top-down) or E-1-t (bottom-up), with
  // off-diagonal b_ie and next diagonal entry a_in; T is loaded eight steps
  // at a time (the stores of the factors would otherwise order every load
  // behind them)
  {
    const int is0 = hb ? E - 1 : 0, ie0 = hb ? E - 2 : 0, in0 = hb ? E - 2 : 1;
    double dcur = dg[is0] - lm;
    if (fabs(dcur) < tiny) dcur = tiny;
    for (int t0 = 0; t0 + 1 < E; t0 += 8) {
      double bo[8], dn[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = (t0 + u + 1 < E) ? t0 + u : t0;  // past the end: a valid row
        bo[u] = od[ie0 + dir * t];
        dn[u] = dg[in0 + dir * t];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        if (t + 1 < E) {  // uniform
          const double x = bo[u] * rcp_acc(dcur);
          own[(is0 + dir * t) * ldz] = x;
          dcur = (dn[u] - lm) - x * bo[u];
          if (fabs(dcur) < tiny) dcur = tiny;
        }
      }
    }
  }
  wave_lds_sync();
  // twist index: lane hb scans i in [lo, hi), downward
  int best = -1;
  double gbest = 0.0;
  {
    const int half = (E + 1) / 2;
    const int lo = hb ? half : 0, hi = hb ? E : half;
    const int n = hi - lo, nmax = E - half > half ? E - half : half;
    for (int t0 = 0; t0 < nmax; t0 += 8) {
      // the operands of eight rows first, then the scan on registers
      double dv[8], zl[8], ol[8], zu[8], ou[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        const int i = hi - 1 - (t < n ? t : 0);
        const int im = i > 0 ? i - 1 : 0, ip = i + 1 < E ? i + 1 : i;
        dv[u] = dg[i];
        zl[u] = zc[im * ldz];
        ol[u] = od[im];
        zu[u] = Z[ip * ldz + b + 32];
        ou[u] = od[i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        const int i = hi - 1 - t;
        double g = dv[u] - lm;
        const double g1 = g - (act ? zl[u] : 0.0) * ol[u];
        g = (i > 0) ? g1 : g;
        const double g2 = g - (act ? zu[u] : 0.0) * ou[u];
        g = (i + 1 < E) ? g2 : g;
        const double ag = fabs(g);
        const bool take = (t < n) & ((best < 0) | (ag < gbest));
        best = take ? i : best;
        gbest = take ? ag : gbest;
      }
    }
  }
  {
    // combine the halves: the upper half wins ties (larger index)
    const int lo_b = __double2loint(gbest), hi_b = __double2hiint(gbest);
    const auto sa = __builtin_amdgcn_permlane32_swap(lo_b, lo_b, false, false);
    const auto sb = __builtin_amdgcn_permlane32_swap(hi_b, hi_b, false, false);
    const auto si = __builtin_amdgcn_permlane32_swap(best, best, false, false);
    // element 0: lower half's values, element 1: upper half's, in every lane
    const double g0 = __hiloint2double(sb[0], sa[0]), g1 = __hiloint2double(sb[1], sa[1]);
    const int b0 = si[0], b1 = si[1];
    best = (b1 >= 0 && (b0 < 0 || g1 <= g0)) ? b1 : b0;
  }
  const int tw = best;
  // outward recurrences from the twist: lane hb = 0 up (z_i = -l_i z_{i+1}),
  // hb = 1 down (z_i = -u_i z_{i-1}); row i = tw - dir (t + 1).  A lane whose
  // steps are done repeats its last value into row tw, which is set to 1
  // afterwards.
  double nrm2 = 0.0;
  {
    const int steps = hb ? (E - 1 - tw) : tw;
    const int smax = (tw > E - 1 - tw) ? tw : E - 1 - tw;
    double zp = 1.0;
    for (int t0 = 0; t0 < smax; t0 += 8) {
      double xs[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        const int i = tw - dir * ((t < steps ? t : -1) + 1);  // 0 <= i < E
        xs[u] = own[i * ldz];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int t = t0 + u;
        if (t < smax) {  // uniform
          const bool on = t < steps;
          const int i = tw - dir * ((on ? t : -1) + 1);
          const double zn = -(act ? xs[u] : 0.0) * zp;
          zp = on ? zn : zp;
          zc[i * ldz] = zp;
          const double n2 = fma(zp, zp, nrm2);
          nrm2 = on ? n2 : nrm2;
        }
      }
    }
  }
  // total squared norm: both halves plus z_tw = 1
  const double tot = sum_halves(nrm2) + 1.0;
  wave_lds_sync();
  if (hb == 0) zc[tw * ldz] = 1.0;
  wave_lds_sync();
  const double inv = rsq_acc(tot);
  if (act) {
    const int half = (E + 1) / 2;
    const int lo = hb ? half : 0, hi = hb ? E : half;
    for (int i0 = lo; i0 < hi; i0 += 8) {
      double zs[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) zs[u] = zc[(i0 + u < hi ? i0 + u : lo) * ldz];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (i0 + u < hi) zc[(i0 + u) * ldz] = zs[u] * inv;
    }
  }
  wave_lds_sync();
}

// Solve (T - mu I) y = b in place (b[i*ldb], i < E) by Gaussian elimination
// with partial pivoting on the tridiagonal matrix (one lane).  Zero pivots
// are replaced by `tiny` (inverse iteration only needs a direction).
// w: 5E doubles of scratch.
template <class MP>
__device__ inline void tridiag_shift_solve(lds_ptr<const double> dg, lds_ptr<const double> od,
                                           int E, double mu, MP b, int ldb, ldsd w, double tiny) {
  ldsd dd = w;           // diagonal of U
  ldsd du = w + E;       // first superdiagonal of U
  ldsd du2 = w + 2 * E;  // second superdiagonal (fill-in from interchanges)
  ldsd ml = w + 3 * E;   // multipliers
  ldsd sw = w + 4 * E;   // 1 where rows i and i+1 were interchanged
  for (int i = 0; i < E; ++i) {
    dd[i] = dg[i] - mu;
    du[i] = (i + 1 < E) ? od[i] : 0.0;
    du2[i] = 0.0;
  }
  for (int i = 0; i + 1 < E; ++i) {
    const double lo = od[i];  // subdiagonal entry below dd[i]
    if (fabs(dd[i]) >= fabs(lo)) {
      const double piv = (dd[i] != 0.0) ? dd[i] : tiny;
      dd[i] = piv;
      const double f = lo / piv;
      ml[i] = f;
      sw[i] = 0.0;
      dd[i + 1] -= f * du[i];
    } else {
      // interchange rows i and i+1, then eliminate
      const double f = dd[i] / lo;
      dd[i] = lo;
      ml[i] = f;
      sw[i] = 1.0;
      const double t = du[i];
      du[i] = dd[i + 1];
      dd[i + 1] = t - f * dd[i + 1];
      if (i + 2 < E) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
    }
  }
  if (dd[E - 1] == 0.0) dd[E - 1] = tiny;
  // forward: row interchanges and L
  for (int i = 0; i + 1 < E; ++i) {
    if (sw[i] == 0.0) {
      b[(i + 1) * ldb] -= ml[i] * b[i * ldb];
    } else {
      const double t = b[i * ldb];
      b[i * ldb] = b[(i + 1) * ldb];
      b[(i + 1) * ldb] = t - ml[i] * b[i * ldb];
    }
  }
  // backward: U
  for (int i = E - 1; i >= 0; --i) {
    double v = b[i * ldb];
    if (i + 1 < E) v -= du[i] * b[(i + 1) * ldb];
    if (i + 2 < E) v -= du2[i] * b[(i + 2) * ldb];
    b[i * ldb] = v / dd[i];
  }
}

// Classical Gram-Schmidt (applied twice) of column j of Z against columns
// 0..j-1 (mutually orthogonal, squared norms cn[c]).  al: >= j doubles.
template <int NT, class MP>
__device__ void cgs2_col(MP Z, int E, int ldz, int j, lds_ptr<const double> cn, ldsd al) {
  const int tid = threadIdx.x;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG16 = NT / 16;
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = g16; c < j; c += NG16) {
      double dt = 0.0;
      for (int i = l16; i < E; i += 16) dt = fma(Z[i * ldz + c], Z[i * ldz + j], dt);
      dt = sum16(dt);
      if (l16 == 0) al[c] = cn[c] > 0.0 ? dt / cn[c] : 0.0;
    }
    __syncthreads();
    for (int i = tid; i < E; i += NT) {
      double v = Z[i * ldz + j];
      for (int c = 0; c < j; ++c) v = fma(-al[c], Z[i * ldz + c], v);
      Z[i * ldz + j] = v;
    }
    __syncthreads();
  }
}

// Squared norm of column j (identical in every 16-lane group).
template <class MP>
__device__ __forceinline__ double col_norm2(MP Z, int E, int ldz, int j) {
  const int l16 = threadIdx.x & 15;
  double s = 0.0;
  for (int i = l16; i < E; i += 16) s = fma(Z[i * ldz + j], Z[i * ldz + j], s);
  return sum16(s);
}

// Modified Gram-Schmidt on columns 0..r-1 of Z (E rows, stride ldz), in
// order.  Column c belongs to the 16-lane group c mod (NT/16), which alone
// updates it; step j removes the (unnormalised) column j from every later
// column, and all columns are normalised at the end.  One barrier per step.
//
// A column that loses most of its norm to the earlier ones came from a
// (numerically) multiple eigenvalue: the twisted factorisation returns the
// same vector for every copy.  It is replaced by inverse iteration with T
// shifted just above lam[j], from a dense start vector kept orthogonal to the
// earlier columns, so the replacement lies in the same eigenspace.  ms: >= kMaxRank + 6 kMaxM doubles.
template <int NT, class MP>
__device__ void mgs_cols(MP Z, int E, int ldz, int r, lds_ptr<const double> dg,
                         lds_ptr<const double> od, lds_ptr<const double> lam, ldsd ms) {
  const int tid = threadIdx.x;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG16 = NT / 16;
  ldsd cn = ms;                     // kMaxRank: squared norms of the finished columns
  ldsd al = ms + kMaxRank;          // kMaxM: projection coefficients / weights
  ldsd lu = al + kMaxM;             // 5 kMaxM: solver scratch
  double tnrm = 0.0;
  for (int i = 0; i < E; ++i)
    tnrm = fmax(tnrm, fabs(dg[i]) + (i > 0 ? fabs(od[i - 1]) : 0.0) + (i + 1 < E ? fabs(od[i]) : 0.0));
  for (int j = 0; j < r; ++j) {
    double s = col_norm2(Z, E, ldz, j);
    if (j > 0 && !(s >= 0.25)) {  // uniform: every group computed the same s
      // dense deterministic start vector (an integer hash of (i, j)), so it
      // has a component in every eigenspace
      for (int i = tid; i < E; i += NT) {
        const unsigned int h = (unsigned int)(i + 1) * 2654435761u ^ (unsigned int)(j + 7) * 40503u;
        Z[i * ldz + j] = (double)(h >> 8) * (1.0 / 8388608.0) - 1.0;
      }
      __syncthreads();
      const double mu = lam[j] + 1e-13 * tnrm;
      for (int it = 0; it < 2; ++it) {
        cgs2_col<NT>(Z, E, ldz, j, cn, al);
        if (tid == 0) tridiag_shift_solve(dg, od, E, mu, Z + j, ldz, lu, 1e-300 + 1e-30 * tnrm);
        __syncthreads();
        const double t = col_norm2(Z, E, ldz, j);
        const double inv = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
        __syncthreads();
        for (int i = tid; i < E; i += NT) Z[i * ldz + j] *= inv;
        __syncthreads();
      }
      cgs2_col<NT>(Z, E, ldz, j, cn, al);
      s = col_norm2(Z, E, ldz, j);
    }
    if (tid == 0) cn[j] = s;
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    for (int c = j + 1 + ((g16 - (j + 1) % NG16 + NG16) % NG16); c < r; c += NG16) {
      double d = 0.0;
      for (int i = l16; i < E; i += 16) d = fma(Z[i * ldz + j], Z[i * ldz + c], d);
      d = sum16(d) * inv;
      for (int i = l16; i < E; i += 16) Z[i * ldz + c] -= d * Z[i * ldz + j];
    }
    __syncthreads();
  }
  for (int c = g16; c < r; c += NG16) {
    double s = 0.0;
    for (int i = l16; i < E; i += 16) s = fma(Z[i * ldz + c], Z[i * ldz + c], s);
    s = sum16(s);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    for (int i = l16; i < E; i += 16) Z[i * ldz + c] *= inv;
  }
  __syncthreads();
}

// Z <- Q Z for the r columns of Z, Q = H_0 H_1 ... H_{E-3} (reflectors in A).
// A 16-lane group owns columns g, g + NT/16, ...; it applies every reflector
// to them in turn (no barrier between reflectors).
template <int NT, class MP, class MPZ>
__device__ void back_transform(MP A, lds_ptr<const double> bt, int E, int lda, MPZ Z,
                               int ldz, int r) {
  const int tid = threadIdx.x;
  const int l16 = tid & 15, g16 = tid >> 4;
  constexpr int NG16 = NT / 16;
  for (int j = E - 3; j >= 0; --j) {
    const double beta = bt[j];
    if (beta == 0.0) continue;  // uniform
    const int m = E - 1 - j;
    const MP v = A + (j + 1) * lda + j;  // v[i*lda], rows j+1..
    for (int c = g16; c < r; c += NG16) {
      double d = 0.0;
      for (int i = l16; i < m; i += 16) d = fma(v[i * lda], Z[(j + 1 + i) * ldz + c], d);
      d = sum16(d) * beta;
      for (int i = l16; i < m; i += 16) Z[(j + 1 + i) * ldz + c] -= d * v[i * lda];
    }
  }
  __syncthreads();
}

}  // namespace qtt

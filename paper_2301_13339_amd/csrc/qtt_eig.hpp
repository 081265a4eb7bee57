// One truncated SVD step of the sweep on the Gram matrix of an unfolding:
// the truncation rule of Algorithm 1 (with the max-rank modification (1)) on
// its eigenvalues, and solve_and_truncate, which runs the eigensolver of
// qtt_syev.hpp, picks the rank and leaves the kept eigenvectors.
#pragma once

#include "qtt_internal.hpp"
#include <type_traits>

#include "qtt_syev.hpp"

namespace qtt {

// Algorithm 1's rule on the sorted eigenvalues of the Gram matrix: smallest
// r >= 1 with sum_{i >= r} lam_i <= tau2 (tails summed from the small end),
// then min(r, cap).  *over is set when the eps-rank exceeded cap.
__device__ inline int truncation_rank_dev(lds_ptr<const double> lam, int E, double tau2, int cap,
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

// The same rule run by one wave: the eigenvalues are loaded into lanes
// (lam[i] in lane i % 64, register i / 64) and read back one at a time in the
// order of truncation_rank_dev, so the sums round identically.  E <= 128.
__device__ inline int truncation_rank_wave(lds_ptr<const double> lam, int E, double tau2, int cap,
                                           int* over) {
  const int l = threadIdx.x & 63;
  const double v0 = (l < E) ? lam[l] : 0.0;
  const double v1 = (l + 64 < E) ? lam[l + 64] : 0.0;
  double tail = 0.0;
  int r = E;
  for (int i = E - 1; i >= 1; --i) {
    const double x = (i < 64) ? v0 : v1;
    const int src = i & 63;
    const double li = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), src),
                                       __builtin_amdgcn_readlane(__double2loint(x), src));
    const double lc = li > 0.0 ? li : 0.0;
    const double t2 = tail + lc;
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

// The rule when only the K = cap largest eigenvalues are known (K < E): the
// tail sums are trace(G) - lam_0 - ... - lam_{r-1}, r = 1..K; when none is
// within tau2 the eps-rank exceeds cap.  One wave; lam[i] in lane i.
__device__ inline int truncation_rank_top(lds_ptr<const double> lam, int K, double trace,
                                          double tau2, int cap, int* over) {
  const int l = threadIdx.x & 63;
  const double v = (l < K) ? lam[l] : 0.0;
  double head = 0.0;
  int r = K + 1;
  for (int i = 0; i < K; ++i) {
    head += __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), i),
                             __builtin_amdgcn_readlane(__double2loint(v), i));
    if (trace - head <= tau2) {
      r = i + 1;
      break;
    }
  }
  *over = r > cap;
  return r < cap ? r : cap;
}

// Singular-value drop-off, modification (3) of Section 5: the smallest
// k >= 1 with sigma_{k+1} < delta sigma_k, i.e. lam[k] < delta^2 lam[k-1]
// on the non-increasing Gram eigenvalues (negative ones read as zero; 0/0 is
// no drop), examined over the K eigenvalues known.  Returns a value above
// every rank when no ratio falls below delta.  One wave.
__device__ inline int dropoff_rank_wave(lds_ptr<const double> lam, int K, double delta2) {
  const int l = threadIdx.x & 63;
  for (int base = 0; base + 1 < K; base += 64) {
    const int i = base + l;
    const bool in = i + 1 < K;  // indices stay below K
    const double a = fmax(lam[in ? i : 0], 0.0), b = fmax(lam[in ? i + 1 : 0], 0.0);
    const bool cut = in & (b < delta2 * a);
    const unsigned long long m = __ballot(cut);
    if (m) return base + __ffsll((unsigned long long)m);  // (first i) + 1
  }
  return 1 << 30;
}

// ----------------------------------------------------- step bookkeeping
// capacities and core offsets, passed by value to the kernels
struct Meta {
  int caps[QTT_MAXD + 1];
  long long offs[QTT_MAXD + 1];
};

struct StepOut {
  int32_t* ranks;
  int32_t* status;
  double* sv;  // may be null
  int lib_capped;
  int32_t* dbg;   // per-step diagnostics in the workspace (optional timings)
  double delta2;  // square of the drop-off threshold of modification (3); 0 = off
};

// Eigen-solve the Gram matrix in A (E x E), choose the rank, and leave the
// kept eigenvectors in the first r columns of V (descending eigenvalues):
// lam[0..E) = eigenvalues in non-increasing order, perm[b] = b.  sx: scratch
// of kEigScratch doubles.  Returns r.  Must be called by all threads.
constexpr int kEigScratch = 10 * kMaxM + 16 + 256;
constexpr int kEigNrmSlot = kEigScratch - 8;  // sx[kEigNrmSlot]: Gershgorin bound of T, [+1]: trace
// one workgroup of 4 waves: a barrier costs ~40 cycles with 4 waves and
// ~470 with 16 on gfx950, and every eigen step is barrier/latency bound
constexpr int kEigThreads = 256;

// Number of eigenvalues of T (diagonal dg, off-diagonal od) below x, by one
// thread: the Sturm sequence of the leading minors of T - xI on T scaled by
// 1 / nrm, rescaled by powers of two every 8 steps (as sturm_counts).
__device__ inline int sturm_below(lds_ptr<const double> dg, lds_ptr<const double> od, int E,
                                  double x, double nrm) {
  const double sc = 1.0 / nrm, xs = x * sc;
  double pm = 1.0, pc = dg[0] * sc - xs;
  int c = sign_change(pc, 1.0);
  for (int i = 1; i < E; ++i) {
    const double b = od[i - 1] * sc;
    const double pn = fma(dg[i] * sc - xs, pc, -fmax(b * b, 1e-60) * pm);
    c += sign_change(pn, pc);
    pm = pc;
    pc = pn;
    if ((i & 7) == 0) {
      const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(pc), fabs(pm)));
      pc = ldexp(pc, -ex);
      pm = ldexp(pm, -ex);
    }
  }
  return c;
}

// Eigenpairs of a symmetric E x E matrix, E = 2 or 4, by cyclic Jacobi in
// one lane on registers (orders this small would spend most of the
// reduction, multisection and twisted factorisation on synchronisation):
// rotations J of (p, q) with tan of twice the angle 2 a_pq / (a_qq - a_pp),
// the smaller root t, A <- J^T A J, V <- V J, sweeps until the off-diagonal
// mass is below 1e-34 of the diagonal's.  la: ascending eigenvalues; V:
// eigenvectors as columns in descending order of eigenvalue.
template <int E, class MP>
__device__ void jacobi_small(MP A, MP V, int lda, ldsd la) {
  double a[E][E], v[E][E];
#pragma unroll
  for (int i = 0; i < E; ++i)
#pragma unroll
    for (int j = 0; j < E; ++j) {
      a[i][j] = 0.5 * (A[i * lda + j] + A[j * lda + i]);
      v[i][j] = (i == j) ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 12; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      dia = fma(a[i][i], a[i][i], dia);
#pragma unroll
      for (int j = i + 1; j < E; ++j) off = fma(a[i][j], a[i][j], off);
    }
    if (!(off > 1e-34 * dia)) break;
#pragma unroll
    for (int p = 0; p < E; ++p)
#pragma unroll
      for (int q = p + 1; q < E; ++q) {
        const double apq = a[p][q];
        if (apq == 0.0) continue;
        // divisions and square roots from the hardware estimates with Newton
        // steps (rcp_acc, rsq_acc): one lane's chain of dependent operations
        const double th = (a[q][q] - a[p][p]) * rcp_acc(2.0 * apq);
        const double th2 = fma(th, th, 1.0);
        const double t = fabs(th) > 1e150 ? 0.5 * rcp_acc(th)
                                          : copysign(1.0, th) * rcp_acc(fabs(th) + th2 * rsq_acc(th2));
        const double c = rsq_acc(fma(t, t, 1.0)), s = t * c;
        a[p][p] -= t * apq;
        a[q][q] += t * apq;
        a[p][q] = a[q][p] = 0.0;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          if (r == p || r == q) continue;
          const double arp = a[r][p], arq = a[r][q];
          a[r][p] = a[p][r] = c * arp - s * arq;
          a[r][q] = a[q][r] = s * arp + c * arq;
        }
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const double vrp = v[r][p], vrq = v[r][q];
          v[r][p] = c * vrp - s * vrq;
          v[r][q] = s * vrp + c * vrq;
        }
      }
  }
  // descending order (selection sort, columns of v with their values)
  double d[E];
#pragma unroll
  for (int i = 0; i < E; ++i) d[i] = a[i][i];
#pragma unroll
  for (int i = 0; i < E; ++i)
#pragma unroll
    for (int j = i + 1; j < E; ++j)
      if (d[j] > d[i]) {
        const double t = d[i];
        d[i] = d[j];
        d[j] = t;
#pragma unroll
        for (int r = 0; r < E; ++r) {
          const double u = v[r][i];
          v[r][i] = v[r][j];
          v[r][j] = u;
        }
      }
#pragma unroll
  for (int i = 0; i < E; ++i) {
    la[E - 1 - i] = d[i];
#pragma unroll
    for (int r = 0; r < E; ++r) V[r * lda + i] = v[r][i];
  }
}

// Whether A - mu I is positive definite (E <= 32), by a Cholesky
// factorisation on the calling wave that stops at the first pivot <= 0: the
// layout of sy_tridiag32w (lane l holds column l & 31, rows 16 (l >> 5) ..),
// the column of step j published in LDS twice, once with rows <= j cleared,
// so the update l_i l_c needs no masks.  A is not modified; rows and
// columns < 32 are read (>= 32 rows allocated, 32 <= lda).  The answer is
// the same in every lane.  buf: >= 64 doubles of LDS private to the wave.
template <class MP>
__device__ bool chol_pd_wave(MP A, int E, int lda, double mu, ldsd buf) {
  const int l = threadIdx.x & 63, c = l & 31, h = l >> 5;
  ldsd colA = buf, colV = buf + 32;
  double a[16];
#pragma unroll
  for (int ii = 0; ii < 16; ++ii) {
    const int r = 16 * h + ii;
    const double t = A[r * lda + c];  // r, c < 32 <= lda
    a[ii] = ((r < E) & (c < E)) ? (r == c ? t - mu : t) : (r == c ? 1.0 : 0.0);
  }
  bool ok = true;
  for (int j = 0; j < E; ++j) {
    if (c == j) {
#pragma unroll
      for (int ii = 0; ii < 16; ++ii) {
        colA[16 * h + ii] = a[ii];
        colV[16 * h + ii] = a[ii];
      }
    }
    if (l <= j) colV[l] = 0.0;  // l <= j <= 31
    wave_lds_sync();
    const double d = colA[j];
    if (!(d > 0.0)) {  // uniform
      ok = false;
      break;
    }
    const double inv = rsq_acc(d);
    const double lc = colV[c] * inv;
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) a[ii] = fma(-colV[16 * h + ii] * inv, lc, a[ii]);
    wave_lds_sync();  // colA, colV are rewritten next step
  }
  wave_lds_sync();  // the next user of buf follows every read above
  return ok;
}

// chol_pd_wave on the first wave, the answer in every thread; flag: one int
// of LDS.  Called by all threads.
template <class MP>
__device__ bool chol_pd32w(MP A, int E, int lda, double mu, ldsd buf, ldsi flag) {
  if (threadIdx.x < 64) {
    const bool ok = chol_pd_wave(A, E, lda, mu, buf);
    if (threadIdx.x == 0) flag[0] = ok ? 1 : 0;
  }
  __syncthreads();
  const bool pd = flag[0] != 0;
  __syncthreads();
  return pd;
}

// try_chol: the caller expects rank E (every earlier step kept full rank), so
// the positive-definiteness test of A - mu I is tried first; when it fails
// (at the pivot of the numerical rank) the usual path decides.
// any_basis: the caller uses only the kept columns of V as a basis (not the
// eigenvalues, and not the vectors as singular vectors).  Then a step whose
// rank is E by the rule (the smallest eigenvalue above tau2, the cap not
// binding, no drop-off cut, no singular values wanted) keeps V = I: the
// step is exact whatever orthonormal basis it keeps, so the eigenvalues and
// vectors are not computed.  One Sturm count at a point a little above tau2
// that finds no eigenvalue below it settles the rank; otherwise the full path
// decides as usual.
template <int NT, bool BIG = false, class MP, class MPV>
__device__ int solve_and_truncate(MP A, MPV V, int E, int lda, ldsd sx, ldsi iscr, ldsd lam,
                                  ldsi perm, double tau2, int cap, int k,
                                  const StepOut& so, bool any_basis = false,
                                  bool try_chol = false) {
  const int tid = threadIdx.x;
  ldsd dg = sx;
  ldsd od = dg + kMaxM;
  ldsd bt = od + kMaxM;
  ldsd pv = bt + kMaxM;
  ldsd e2 = pv + kMaxM;
  ldsd la = e2 + kMaxM;  // ascending eigenvalues
  // the tridiagonalisation takes pv .. pv + 4 kMaxM (over e2 and la, which are
  // used only after it) for its column and p buffers
  // finiteness of the Gram (NaN/Inf input): its trace, by wave 0
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < E; i += 64) tr += A[i * lda + i];
    tr = sum64(tr);
    if (tid == 0) {
      iscr[1] = isfinite(tr) ? 1 : 0;
      sx[kEigNrmSlot + 1] = tr;
    }
  }
  __syncthreads();
  const int finite = iscr[1];
#ifdef QTT_EIG_TIMING
  long long tt[6];
  tt[0] = wall_clock64();
#endif
  double tnrm = 0.0;  // Gershgorin bound of T
  // orders 2 and 4: every eigenpair by jacobi_small
  const bool small = std::is_same<MP, MPV>::value && finite && (E == 2 || E == 4);
  // eigenvalues computed: all when the singular values are reported, the cap
  // does not bind or the tolerance is zero, else the cap largest (the rank
  // rule then works from the trace)
  const int K = (small || so.sv || cap >= E || !(tau2 > 0.0)) ? E : cap;
  // rank E by the rule (any basis then serves): decided before any reduction
  // when A - mu I is positive definite, mu a little above tau2
  auto keep_all = [&]() {
    for (int i = tid; i < E; i += NT) {
      lam[i] = 0.0;
      perm[i] = i;
    }
    for (int idx = tid; idx < E * E; idx += NT) {
      const int a = idx / E, c = idx - a * E;
      V[a * lda + c] = (a == c) ? 1.0 : 0.0;
    }
    if (tid == 0) {
      iscr[2] = E;
      so.ranks[k] = E;
    }
    __syncthreads();
  };
  const bool full_test = any_basis && !so.sv && !(so.delta2 > 0.0) && cap >= E;
  if (try_chol && finite && !small && full_test && E <= 32 &&
      chol_pd32w(A, E, lda, tau2 * (1.0 + 1e-6) + 1e-12 * sx[kEigNrmSlot + 1], pv, iscr + 4)) {
    keep_all();
    return E;
  }
  if (small) {
    if constexpr (std::is_same<MP, MPV>::value) {
      if (tid == 0) {
        if (E == 2)
          jacobi_small<2>(A, V, lda, la);
        else
          jacobi_small<4>(A, V, lda, la);
      }
    }
    __syncthreads();
  } else if (finite) {
    if constexpr (BIG) {
      // the E <= 64 reduction leaves Q^T in A, which the back transformation
      // of split storage (A and V in different memories) does not take
      if (E > 64 || !std::is_same<MP, MPV>::value)
        sy_tridiag<NT, 8>(A, E, lda, dg, od, bt, pv);
      else if (E <= 16)
        sy_tridiag16w(A, E, lda, dg, od, bt, pv);
      else if (E <= 32)
        sy_tridiag32w(A, E, lda, dg, od, bt, pv);
      else
        sy_tridiag64(A, E, lda, dg, od, bt, pv);
    } else {
      if (E <= 16)
        sy_tridiag16w(A, E, lda, dg, od, bt, pv);
      else if (E <= 32)
        sy_tridiag32w(A, E, lda, dg, od, bt, pv);
      else
        sy_tridiag64(A, E, lda, dg, od, bt, pv);
    }
#ifdef QTT_EIG_TIMING
    tt[1] = wall_clock64();
#endif
    tnrm = tridiag_gersh(dg, od, E, sx + kEigNrmSlot);
    if (full_test && E > 32 && tnrm > 0.0) {
      if (tid == 0) iscr[4] = sturm_below(dg, od, E, tau2 * (1.0 + 1e-6) + 1e-12 * tnrm, tnrm);
      __syncthreads();
      if (iscr[4] == 0) {  // uniform: rank E, any orthonormal basis
        keep_all();
        return E;
      }
    }
    tridiag_eigvals<NT>(dg, od, E, la, e2, pv, tnrm, K);
  }
#ifdef QTT_EIG_TIMING
  tt[2] = wall_clock64();
#endif
  for (int i = tid; i < E; i += NT) {
    lam[i] = (finite && i < K) ? la[E - 1 - i] : 0.0;
    perm[i] = i;
  }
  __syncthreads();
  if (tid < 64) {
    int over = 0;
    int r = (K < E) ? truncation_rank_top(lam, K, sx[kEigNrmSlot + 1], tau2, cap, &over)
                    : truncation_rank_wave(lam, E, tau2, cap, &over);
    if (so.delta2 > 0.0 && finite) {
      // the drop-off cut; a cut within the cap means the cap did not decide
      const int rd = dropoff_rank_wave(lam, K, so.delta2);
      if (rd < r) r = rd;
      if (rd <= cap) over = 0;
    }
    if (tid == 0) {
      iscr[2] = r;
      so.ranks[k] = r;
      if (so.status) {
        if (!finite) atomicOr(so.status, QTT_STATUS_NONFINITE);
        if (over && so.lib_capped) atomicOr(so.status, QTT_STATUS_RANKCAP);
      }
    }
  }
  if (so.sv) {
    for (int i = tid; i < kSvStride; i += NT) {
      const double l = (i < E) ? lam[i] : 0.0;
      so.sv[(size_t)(k - 1) * kSvStride + i] = l > 0.0 ? sqrt(l) : 0.0;
    }
  }
  __syncthreads();
  const int r = iscr[2];
  if (small) {  // V holds every eigenvector, in order
#ifdef QTT_EIG_TIMING
    if (tid == 0 && so.dbg) {
      so.dbg[k] = E;
      int* t5 = so.dbg + 64 + 5 * k;
      t5[0] = 0;
      t5[1] = (int)(wall_clock64() - tt[0]);
      t5[2] = t5[3] = t5[4] = 0;
    }
#endif
    return r;
  }
  if (!finite) {
    for (int idx = tid; idx < E * E; idx += NT) {
      const int a = idx / E, c = idx - a * E;
      V[a * lda + c] = (a == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    return r;
  }
  // eigenvectors of T for the kept eigenvalues, one lane per vector
  {
    const double tiny = 1e-300 + 1e-30 * tnrm;
    if (E <= 64 && r <= 32) {
      if (tid < 64) tridiag_vec_pair(dg, od, E, lam, V, lda, r, tiny);
    } else {
      for (int b = tid; b < r; b += NT) tridiag_vec(dg, od, E, lam[b], V + b, lda, tiny);
    }
  }
  __syncthreads();
#ifdef QTT_EIG_TIMING
  tt[3] = wall_clock64();
#endif
  // pv .. sx + kEigNrmSlot (pv, e2, la and the arrays after) are free now
  bool small_done = false;
  if constexpr (std::is_same<MP, MPV>::value) {
    if (E <= 64) {
      // A holds Q^T of the reduction (sy_tridiag64); vectors that are
      // orthonormal to first order take one polishing step, others (or more
      // than 32) Gram-Schmidt
      const bool done = (r <= 32 && polish_backtr64(A, E, lda, V, r, pv)) ||
                        (r > 32 && polish_backtr64_wide(A, E, lda, V, r, pv)) ||
                        mgs_backtr64(A, E, lda, V, lda, r, pv, iscr + 3);
#ifdef QTT_EIG_TIMING
      tt[4] = wall_clock64();
#endif
      if (!done) {
        mgs_cols<NT>(V, E, lda, r, dg, od, lam, pv);
        backtr_gemm64(A, E, lda, V, r);
      }
      small_done = true;
    }
  }
  if (!small_done) {
    mgs_cols<NT>(V, E, lda, r, dg, od, lam, pv);
#ifdef QTT_EIG_TIMING
    tt[4] = wall_clock64();
#endif
    back_transform<NT>(A, bt, E, lda, V, lda, r);
  }
#ifdef QTT_EIG_TIMING
  tt[5] = wall_clock64();
  if (tid == 0 && so.dbg) {
    so.dbg[k] = E;
    int* tm = so.dbg + 64 + 4 * k;
    (void)tm;
    int* t5 = so.dbg + 64 + 5 * k;
    t5[0] = (int)(tt[1] - tt[0]);
    t5[1] = (int)(tt[2] - tt[1]);
    t5[2] = (int)(tt[3] - tt[2]);
    t5[3] = (int)(tt[4] - tt[3]);
    t5[4] = (int)(tt[5] - tt[4]);
  }
#endif
  return r;
}

}  // namespace qtt

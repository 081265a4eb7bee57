// QTT convolution (exact Toeplitz operator in QTT-matrix form) and Full
// (Algorithm 3) on gfx950.
#include "qtt_internal.hpp"

namespace qtt {

// ====================================================================== conv
// The discrete convolution (2.2) on one axis of N = 2^d samples is
// y_j = sum_i w_{j-i+N} f_i.  Write u = j + ibar + 1 with ibar = N-1-i (the
// bitwise complement of i): u is a binary addition with carry-in 1, so bit k
// of u is (j_k + 1 - i_k + c_{k-1}) mod 2 and the carry c_k is its quotient;
// u_{d+1} = c_d.  With w in QTT form (d+1 modes, cores W_1..W_{d+1}) the
// operator T(j,i) = w_u is a QTT matrix whose core k has bond (kernel bond,
// carry): T_k[(a,c), j, i, (a',c')] = W_k[a, u_k, a'] [c' = carry], the
// carry-in of the first core is 1 and the last core absorbs W_{d+1}[., c_d, 0].
// The product with the signal cores F_k gives the output cores
// Y_k[(a,c,b), j, (a',c',b')] = sum_i T_k[(a,c), j, i, (a',c')] F_k[b, i, b'].
// An image (row-major) has the column axis on modes 1..dx and the row axis
// on modes dx+1..dx+dy; the bond between the two axes is the signal bond.

struct ConvMode {
  int axis;       // axis index of this mode
  int kappa;      // 1-based position within the axis
  int last;       // 1 if kappa == d_axis (closing core)
};

struct ConvMeta {
  ConvMode mode[QTT_MAXD];
  long long yoff[QTT_MAXD + 1];
  long long foff[QTT_MAXD + 1];
  long long woff[2][QTT_MAXD + 2];
  int32_t* wranks[2];
  const void* wcores[2];
  int dax[2];
};

template <typename T>
__global__ void k_conv_cores(const T* fcores, const int32_t* franks, ConvMeta cm, T* ycores,
                             int32_t* yranks, long long max_elems, int d) {
  const int k = blockIdx.y;  // 0-based mode
  const ConvMode md = cm.mode[k];
  const int32_t* wr = cm.wranks[md.axis];
  const T* W = static_cast<const T*>(cm.wcores[md.axis]);
  const int kap = md.kappa;                 // 1-based
  const int rho0 = wr[kap - 1], rho1 = wr[kap];
  const int f0 = franks[k], f1 = franks[k + 1];
  const int L = (kap == 1) ? f0 : 2 * rho0 * f0;
  const int R = md.last ? f1 : 2 * rho1 * f1;
  const long long total = (long long)L * 2 * R;
  const T* Fk = fcores + cm.foff[k];
  const T* Wk = W + cm.woff[md.axis][kap - 1];
  const T* Wl = W + cm.woff[md.axis][kap];  // W_{d+1} when last
  const int rhol = md.last ? wr[kap + 1] : 0;  // == 1
  (void)rhol;
  T* Yk = ycores + cm.yoff[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    yranks[k + 1] = (k + 1 == d) ? 1 : R;
    if (k == 0) yranks[0] = 1;
  }
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int col = (int)(e % R);
    const long long rj = e / R;
    const int j = (int)(rj & 1);
    const int row = (int)(rj >> 1);
    // left bond (a, c, b)
    int a, c, b;
    if (kap == 1) {
      a = 0;
      c = 1;
      b = row;
    } else {
      b = row % f0;
      const int ac = row / f0;
      c = ac & 1;
      a = ac >> 1;
    }
    double acc = 0.0;
    if (!md.last) {
      const int b1 = col % f1;
      const int ac1 = col / f1;
      const int c1 = ac1 & 1, a1 = ac1 >> 1;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int v = j + (1 - i) + c;
        if ((v >> 1) != c1) continue;
        const int u = v & 1;
        const double wv = (double)Wk[((long long)a * 2 + u) * rho1 + a1];
        const double fv = (double)Fk[((long long)b * 2 + i) * f1 + b1];
        acc += wv * fv;
      }
    } else {
      const int b1 = col;  // closing: right bond is the signal bond only
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int v = j + (1 - i) + c;
        const int u = v & 1, cr = v >> 1;
        double t = 0.0;
        for (int a1 = 0; a1 < rho1; ++a1)
          t += (double)Wk[((long long)a * 2 + u) * rho1 + a1] * (double)Wl[a1 * 2 + cr];
        acc += t * (double)Fk[((long long)b * 2 + i) * f1 + b1];
      }
    }
    Yk[e] = (T)acc;
  }
}

int run_conv(const TensorDev& f, const TensorDev* w, int n_axes, const int32_t* axis_modes,
             const TensorDev& y, int dtype, hipStream_t stream) {
  ConvMeta cm;
  int k = 0;
  for (int a = 0; a < n_axes; ++a) {
    cm.dax[a] = axis_modes[a];
    cm.wranks[a] = w[a].ranks;
    cm.wcores[a] = w[a].cores;
    for (int j = 0; j <= w[a].d; ++j) cm.woff[a][j] = w[a].off[j];
    for (int kap = 1; kap <= axis_modes[a]; ++kap, ++k) {
      cm.mode[k].axis = a;
      cm.mode[k].kappa = kap;
      cm.mode[k].last = (kap == axis_modes[a]);
    }
  }
  for (int j = 0; j <= f.d; ++j) {
    cm.yoff[j] = y.off[j];
    cm.foff[j] = f.off[j];
  }
  long long maxe = 0;
  for (int j = 0; j < f.d; ++j) {
    const long long e = (long long)y.cap[j] * 2 * y.cap[j + 1];
    if (e > maxe) maxe = e;
  }
  long long bx = (maxe + 255) / 256;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  dim3 grid((unsigned)bx, (unsigned)f.d);
  ProbeScope _ps(QTT_K_CONV, stream);
  if (dtype == QTT_F64) {
    k_conv_cores<double><<<grid, 256, 0, stream>>>(static_cast<const double*>(f.cores), f.ranks,
                                                   cm, static_cast<double*>(y.cores), y.ranks,
                                                   maxe, f.d);
  } else {
    k_conv_cores<float><<<grid, 256, 0, stream>>>(static_cast<const float*>(f.cores), f.ranks, cm,
                                                  static_cast<float*>(y.cores), y.ranks, maxe,
                                                  f.d);
  }
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

// ====================================================================== full
// Algorithm 3 reorganised as two half chains and one product.  With the left
// modes 1..m and the right modes m+1..d,
//   Lam_k (2^k x r_k):       Lam_k[lo + 2^(k-1) i, b] = sum_a Lam_{k-1}[lo, a] G_k[a, i, b]
//   Rho_k (r_{k-1} x 2^(d-k+1)): Rho_k[a, i + 2 hi] = sum_b G_k[a, i, b] Rho_{k+1}[b, hi]
//   out[lo + 2^m hi] = sum_a Lam_m[lo, a] Rho_{m+1}[a, hi].
// Each is a tiled product C = A B (A: M x K, B: K x N row-major) whose
// result is scattered by the layout of the mode.
enum { GEMM_LEFT = 0, GEMM_RIGHT = 1, GEMM_FINAL = 2 };

// Chain products on the matrix cores: v_mfma_f64_16x16x4f64 (FP64) and
// v_mfma_f32_16x16x4f32 (FP32, FP32 accumulation) take one A entry per lane
// (row l % 16, k = l / 16) and one B entry (k = l / 16, column l % 16); the
// FP64 instruction leaves D[4i + l / 16][l % 16] in accumulator i, the FP32
// one D[4 (l / 16) + i][l % 16].  A workgroup of four waves owns a
// tile of C (32 x 32: one 16 x 16 block per wave, which keeps several
// workgroups per compute unit for the narrow chains of Full); the A and B
// panels of TK k-values pass through LDS (stored k-major, so the fragment
// reads of a wave are 16 consecutive elements per k).
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  using type = f64x4;
  static __device__ __forceinline__ f64x4 step(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 block held by accumulator e of lane l
  static __device__ __forceinline__ int row(int e, int l) { return 4 * e + (l >> 4); }
};
template <>
struct MfmaAcc<float> {
  using type = f32x4;
  static __device__ __forceinline__ f32x4 step(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int e, int l) { return 4 * (l >> 4) + e; }
};

template <typename T, int MODE, int SZ, int TK>
__device__ __forceinline__ void chain_tile(const T* A, const T* B, T* C, const int32_t* ranks,
                                           int k, int Mh, int Nh, int bx, int by,
                                           T (*As)[TK][SZ + 4], T (*Bs)[TK][SZ + 4]) {
  using acc_t = typename MfmaAcc<T>::type;
  // SZ x SZ tile (bx, by) per workgroup; each wave an (SZ/2) x (SZ/2)
  // quarter made of NB x NB blocks of 16 x 16
  constexpr int NB = SZ / 32, PA = SZ * TK / 256;
  int M, N, K, rk = 0;
  if (MODE == GEMM_LEFT) {
    K = ranks[k - 1];
    rk = ranks[k];
    M = Mh;
    N = 2 * rk;
  } else if (MODE == GEMM_RIGHT) {
    M = 2 * ranks[k - 1];
    K = ranks[k];
    N = Nh;
  } else {
    M = Mh;
    K = ranks[k];
    N = Nh;
  }
  const int row0 = by * SZ, col0 = bx * SZ;
  if (row0 >= M || col0 >= N) return;  // uniform
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int wr = (w >> 1) * (SZ / 2), wc = (w & 1) * (SZ / 2);
  // global -> LDS assignment: A panel SZ rows x TK k (PA consecutive k per
  // thread), B panel TK k x SZ columns (PA consecutive columns per thread)
  const int am = tid / (TK / PA), ak = (tid % (TK / PA)) * PA;
  const int bk = tid / (SZ / PA), bn = (tid % (SZ / PA)) * PA;
  T ra[PA], rb[PA];
  auto load = [&](int k0) {
    const int gr = row0 + am;
#pragma unroll
    for (int t = 0; t < PA; ++t) {
      const int gk = k0 + ak + t;
      ra[t] = (gr < M && gk < K) ? A[(long long)gr * K + gk] : (T)0;
    }
    const int gk = k0 + bk;
#pragma unroll
    for (int t = 0; t < PA; ++t) {
      const int gc = col0 + bn + t;
      rb[t] = (gk < K && gc < N) ? B[(long long)gk * N + gc] : (T)0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int t = 0; t < PA; ++t) As[buf][ak + t][am] = ra[t];
#pragma unroll
    for (int t = 0; t < PA; ++t) Bs[buf][bk][bn + t] = rb[t];
  };
  acc_t acc[NB][NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = acc_t{(T)0, (T)0, (T)0, (T)0};
  const int nk = (K + TK - 1) / TK;
  load(0);
  store(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load((kt + 1) * TK);  // global loads in flight during the products
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      const int kr = kk + (l >> 4);
      T fa[NB], fb[NB];
#pragma unroll
      for (int i = 0; i < NB; ++i) fa[i] = As[cur][kr][wr + 16 * i + (l & 15)];
#pragma unroll
      for (int j = 0; j < NB; ++j) fb[j] = Bs[cur][kr][wc + 16 * j + (l & 15)];
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = MfmaAcc<T>::step(fa[i], fb[j], acc[i][j]);
    }
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gr = row0 + wr + 16 * i + MfmaAcc<T>::row(e, l);
        const int gc = col0 + wc + 16 * j + (l & 15);
        if (gr >= M || gc >= N) continue;
        long long dst;
        if (MODE == GEMM_LEFT) {
          const int ii = gc / rk, bb = gc - ii * rk;
          dst = ((long long)gr + (long long)Mh * ii) * rk + bb;
        } else if (MODE == GEMM_RIGHT) {
          dst = (long long)(gr >> 1) * (2LL * N) + (gr & 1) + 2LL * gc;
        } else {
          dst = (long long)gr + (long long)M * gc;
        }
        C[dst] = acc[i][j][e];
      }
}

template <typename T, int MODE, int SZ, int TK>
__global__ void __launch_bounds__(256) k_chain_mfma(const T* A, const T* B, T* C,
                                                    const int32_t* ranks, int k, int Mh, int Nh) {
  __shared__ T As[2][TK][SZ + 4];
  __shared__ T Bs[2][TK][SZ + 4];
  chain_tile<T, MODE, SZ, TK>(A, B, C, ranks, k, Mh, Nh, blockIdx.x, blockIdx.y, As, Bs);
}

// One step of the left chain and one of the right chain in a single launch
// (they are independent until the final product): blocks 0 .. glx*gly - 1
// take the left step's tiles, the rest the right step's.
template <typename T, int SZ, int TK>
__global__ void __launch_bounds__(256) k_chain_pair(const T* lamA, const T* coreL, T* dstL, int kl,
                                                    int Mh, int glx, int gly, const T* coreR,
                                                    const T* rhoB, T* dstR, int kr, int Nh,
                                                    int grx, const int32_t* ranks) {
  __shared__ T As[2][TK][SZ + 4];
  __shared__ T Bs[2][TK][SZ + 4];
  const int b = blockIdx.x, nl = glx * gly;
  if (b < nl)
    chain_tile<T, GEMM_LEFT, SZ, TK>(lamA, coreL, dstL, ranks, kl, Mh, 0, b % glx, b / glx, As,
                                     Bs);
  else
    chain_tile<T, GEMM_RIGHT, SZ, TK>(coreR, rhoB, dstR, ranks, kr, 0, Nh, (b - nl) % grx,
                                      (b - nl) / grx, As, Bs);
}

// d == 1: out = core
template <typename T>
__global__ void k_copy_single(const T* core, T* out) {
  if (threadIdx.x < 2) out[threadIdx.x] = core[threadIdx.x];
}

static void full_sizes(int d, const int32_t* cap, int* m, size_t* lam_elems, size_t* rho_elems) {
  *m = d / 2;
  size_t le = 2, re = 2;
  for (int k = 1; k <= *m; ++k) {
    const size_t e = ((size_t)1 << k) * (size_t)cap[k];
    if (e > le) le = e;
  }
  for (int k = d; k > *m; --k) {
    const size_t e = (size_t)cap[k - 1] * ((size_t)1 << (d - k + 1));
    if (e > re) re = e;
  }
  *lam_elems = le;
  *rho_elems = re;
}

int plan_full(int d, const int32_t* cap, int dtype, void* ws, size_t* ws_bytes, void** bufs) {
  int m;
  size_t le, re;
  full_sizes(d, cap, &m, &le, &re);
  Arena ar(ws);
  const size_t es = elem_size(dtype);
  bufs[0] = ar.take<char>(le * es);
  bufs[1] = ar.take<char>(le * es);
  bufs[2] = ar.take<char>(re * es);
  bufs[3] = ar.take<char>(re * es);
  if (ws_bytes) *ws_bytes = ar.size();
  return QTT_OK;
}

template <typename T>
static int run_full_t(const TensorDev& t, T* out, void* ws, hipStream_t stream) {
  const int d = t.d;
  const T* cores = static_cast<const T*>(t.cores);
  if (d == 1) {
    {
      ProbeScope _ps(QTT_K_OTHER, stream);
      k_copy_single<T><<<1, 64, 0, stream>>>(cores, out);
    }
    QTT_LAUNCH_CHECK();
    return QTT_OK;
  }
  int32_t cap[QTT_MAXD + 1];
  for (int k = 0; k <= d; ++k) cap[k] = t.cap[k];
  void* bufs[4];
  size_t wsb = 0;
  plan_full(d, cap, sizeof(T) == 8 ? QTT_F64 : QTT_F32, ws, &wsb, bufs);
  int m;
  size_t le, re;
  full_sizes(d, cap, &m, &le, &re);
  // left chain: Lam_1 = core 1 memory (2 x r_1); right chain: Rho_d = core d
  // memory (r_{d-1} x 2).  The two chains advance together, one launch per
  // pair of steps.
  const T* lam = cores + t.off[0];
  int li = 0;
  const T* rho = cores + t.off[d - 1];
  int ri = 2;
  int kl = 2, kr = d - 1;
  {
    for (; kl <= m && kr >= m + 1; ++kl, --kr) {
      T* dl = static_cast<T*>(bufs[li]);
      T* dr = static_cast<T*>(bufs[ri]);
      const int Mh = 1 << (kl - 1), Nh = 1 << (d - kr);
      const int glx = (2 * cap[kl] + 31) / 32, gly = (Mh + 31) / 32;
      const int grx = (Nh + 31) / 32, gry = (2 * cap[kr - 1] + 31) / 32;
      {
        ProbeScope _ps(QTT_K_FULL_CHAIN, stream);
        k_chain_pair<T, 32, 32><<<glx * gly + grx * gry, 256, 0, stream>>>(
            lam, cores + t.off[kl - 1], dl, kl, Mh, glx, gly, cores + t.off[kr - 1], rho, dr, kr,
            Nh, grx, t.ranks);
      }
      QTT_LAUNCH_CHECK();
      lam = dl;
      li ^= 1;
      rho = dr;
      ri = ri == 2 ? 3 : 2;
    }
  }
  for (int k = kl; k <= m; ++k) {
    T* dst = static_cast<T*>(bufs[li]);
    const int Mh = 1 << (k - 1);
    const int Ncap = 2 * cap[k];
    const int ts = 32;  // tile of the matrix-core kernel
    dim3 grid((Ncap + ts - 1) / ts, (Mh + ts - 1) / ts);
    {
      ProbeScope _ps(QTT_K_FULL_CHAIN, stream);
      k_chain_mfma<T, GEMM_LEFT, 32, 32><<<grid, 256, 0, stream>>>(lam, cores + t.off[k - 1], dst,
                                                                   t.ranks, k, Mh, 0);
    }
    QTT_LAUNCH_CHECK();
    lam = dst;
    li ^= 1;
  }
  for (int k = kr; k >= m + 1; --k) {
    T* dst = static_cast<T*>(bufs[ri]);
    const int Nh = 1 << (d - k);
    const int Mcap = 2 * cap[k - 1];
    const int ts = 32;
    dim3 grid((Nh + ts - 1) / ts, (Mcap + ts - 1) / ts);
    {
      ProbeScope _ps(QTT_K_FULL_CHAIN, stream);
      k_chain_mfma<T, GEMM_RIGHT, 32, 32><<<grid, 256, 0, stream>>>(cores + t.off[k - 1], rho,
                                                                    dst, t.ranks, k, 0, Nh);
    }
    QTT_LAUNCH_CHECK();
    rho = dst;
    ri = ri == 2 ? 3 : 2;
  }
  {
    const int Mh = 1 << m, Nh = 1 << (d - m);
    const int ts = 32;
    dim3 grid((Nh + ts - 1) / ts, (Mh + ts - 1) / ts);
    {
      ProbeScope _ps(QTT_K_FULL_FINAL, stream);
      k_chain_mfma<T, GEMM_FINAL, 32, 32><<<grid, 256, 0, stream>>>(lam, rho, out, t.ranks, m, Mh,
                                                                    Nh);
    }
    QTT_LAUNCH_CHECK();
  }
  return QTT_OK;
}

int run_full(const TensorDev& t, int dtype, void* out, void* ws, hipStream_t stream) {
  if (dtype == QTT_F64) return run_full_t<double>(t, static_cast<double*>(out), ws, stream);
  return run_full_t<float>(t, static_cast<float*>(out), ws, stream);
}

}  // namespace qtt

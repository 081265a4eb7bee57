// Adjoint of the convolution + reconstruction on gfx950.
//
// Loss-independent pieces of the backward of y = T(w) full(F), where T(w)
// is the Toeplitz form of the discrete convolution (2.2) with generator w
// (a QTT with d+1 modes, the sinc kernel (3.1)/(7.2)) and full(F) the
// reconstruction of Algorithm 3:
//   * toeplitz_apply: y = T(w) x or x = T(w)^T y for full vectors, with the
//     operator in its QTT-matrix (MPO) form -- the binary adder
//     u = j + ibar + 1 with carry (the same operator as qtt_conv);
//   * full_adjoint: the gradient of <g, full(F)> with respect to every core,
//     from the right interfaces of F (recomputed here, never stored by the
//     forward) and the left partial contractions of g;
//   * the bandwidth derivative: dL/dB = <grad_y, T(dw/dB) full(F)> with
//     dw/dB in QTT form (generated on the device, decomposed by the sweep).
#include <math.h>
#include <string.h>

#include <mutex>

#include "qtt_internal.hpp"
#include "qtt_sinc.hpp"

namespace qtt {

// ===================================================== Toeplitz MPO, full
// State after step k (bits 1..k processed): S_k[b][pos], b = 2 alpha + c
// (kernel bond alpha < rho_k, carry c), pos < N.  In a forward product the
// bits 1..k of pos are output bits j and the others input bits i; in a
// transposed product the roles swap.  One step consumes bit k:
//   S_k[(a',c')][..o..] = sum_{a,c,n} [c' = carry] W_k[a, u, a'] S_{k-1}[(a,c)][..n..]
// with (j, i) = (o, n) (forward) or (n, o) (transposed), v = j + (1-i) + c,
// u = v mod 2 and carry = v div 2.  S_0 = x with alpha = 0 and carry-in 1;
// the last step contracts u_{d+1} = c_d with W_{d+1}.
struct ToepMeta {
  long long woff[QTT_MAXD + 2];  // element offsets of the w cores
};

__device__ __forceinline__ long long ins_bit(long long q, int bit, int v) {
  const long long lo = q & ((1LL << bit) - 1);
  return lo | ((long long)v << bit) | ((q >> bit) << (bit + 1));
}

constexpr int kToepNB = 8;  // output bonds per thread (for both output bits)

// middle and first steps (not the last)
// TI: element type of the input (the caller's x on the first step, else the
// FP64 state); the state is always FP64, T is the type of the w cores
template <typename T, typename TI, int TRANS, int FIRST>
__global__ void __launch_bounds__(256) k_toep_step(const TI* in, double* out, const T* wc,
                                                   const int32_t* wr, ToepMeta tm, int k,
                                                   long long N) {
  const long long half = N >> 1;
  const long long q = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  const int rin = FIRST ? 1 : wr[k - 1];
  const int rout = wr[k];
  const int b0 = (blockIdx.y * 4 + w) * kToepNB;  // first output bond of this thread
  if (b0 >= 2 * rout || q >= half) return;
  const T* Wk = wc + tm.woff[k - 1];  // W_k[a][u][a'] at (a*2 + u)*rout + a'
  const int bit = k - 1;
  const long long p0 = ins_bit(q, bit, 0), p1 = ins_bit(q, bit, 1);
  double acc[kToepNB][2];
#pragma unroll
  for (int t = 0; t < kToepNB; ++t) acc[t][0] = acc[t][1] = 0.0;
  for (int a = 0; a < rin; ++a) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (FIRST && c == 0) continue;  // carry-in is 1
      const long long row = FIRST ? 0 : (long long)(2 * a + c) * N;
      const double x0 = (double)in[row + p0], x1 = (double)in[row + p1];
#pragma unroll
      for (int t = 0; t < kToepNB; ++t) {
        const int bo = b0 + t;
        if (bo < 2 * rout) {
          const int a1 = bo >> 1, c1 = bo & 1;
#pragma unroll
          for (int o = 0; o < 2; ++o) {
#pragma unroll
            for (int n = 0; n < 2; ++n) {
              const int jb = TRANS ? n : o, ib = TRANS ? o : n;
              const int v = jb + (1 - ib) + c;
              if ((v >> 1) == c1) {
                const double wv = (double)Wk[(a * 2 + (v & 1)) * rout + a1];
                acc[t][o] = fma(wv, n ? x1 : x0, acc[t][o]);
              }
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kToepNB; ++t) {
    const int bo = b0 + t;
    if (bo < 2 * rout) {
      out[(long long)bo * N + p0] = acc[t][0];
      out[(long long)bo * N + p1] = acc[t][1];
    }
  }
}

// last step (k = d): y[pos] = sum_{a,c,n} V[a][u][c'] S_{d-1}[(a,c)][pos_n] with
// V[a][u][c'] = sum_{a'} W_d[a, u, a'] W_{d+1}[a', c', 0]
template <typename T, typename TI, int TRANS, int FIRST>
__global__ void __launch_bounds__(256) k_toep_last(const TI* in, T* y, const T* wc,
                                                   const int32_t* wr, ToepMeta tm, int d,
                                                   long long N) {
  __shared__ double V[kMaxRank * 4];
  const int rin = FIRST ? 1 : wr[d - 1];
  const int rmid = wr[d];
  const T* Wd = wc + tm.woff[d - 1];
  const T* Wl = wc + tm.woff[d];  // (rmid, 2, 1)
  for (int e = threadIdx.x; e < rin * 4; e += blockDim.x) {
    const int a = e >> 2, u = (e >> 1) & 1, c1 = e & 1;
    double s = 0.0;
    for (int a1 = 0; a1 < rmid; ++a1)
      s = fma((double)Wd[(a * 2 + u) * rmid + a1], (double)Wl[a1 * 2 + c1], s);
    V[e] = s;
  }
  __syncthreads();
  const long long half = N >> 1;
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= half) return;
  const int bit = d - 1;
  const long long p0 = ins_bit(q, bit, 0), p1 = ins_bit(q, bit, 1);
  double y0 = 0.0, y1 = 0.0;
  for (int a = 0; a < rin; ++a) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (FIRST && c == 0) continue;
      const long long row = FIRST ? 0 : (long long)(2 * a + c) * N;
      const double x0 = (double)in[row + p0], x1 = (double)in[row + p1];
#pragma unroll
      for (int o = 0; o < 2; ++o) {
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          const int jb = TRANS ? n : o, ib = TRANS ? o : n;
          const int v = jb + (1 - ib) + c;
          const double t = V[a * 4 + (v & 1) * 2 + (v >> 1)] * (n ? x1 : x0);
          if (o)
            y1 += t;
          else
            y0 += t;
        }
      }
    }
  }
  y[p0] = (T)y0;
  y[p1] = (T)y1;
}

// FP64 elements of the two state buffers
size_t toeplitz_ws_elems(int d, const int32_t* w_cap) {
  int rmax = 1;
  for (int k = 1; k < d; ++k) rmax = w_cap[k] > rmax ? w_cap[k] : rmax;
  return 2 * (size_t)(2 * rmax) * ((size_t)1 << d);
}

template <typename T>
static int toeplitz_t(const TensorDev& w, const T* x, T* y, int trans, double* ws,
                      hipStream_t s) {
  const int d = w.d - 1;
  const long long N = 1LL << d;
  ToepMeta tm;
  for (int k = 0; k <= w.d; ++k) tm.woff[k] = w.off[k];
  const T* wc = static_cast<const T*>(w.cores);
  int rmax = 1;
  for (int k = 1; k < d; ++k) rmax = w.cap[k] > rmax ? w.cap[k] : rmax;
  double* buf[2] = {ws, ws + (size_t)(2 * rmax) * N};
  const long long half = N >> 1;
  ProbeScope _ps(QTT_K_ADJOINT, s);
  const unsigned gl = (unsigned)((half + 255) / 256);
  if (d == 1) {
    if (trans)
      k_toep_last<T, T, 1, 1><<<gl, 256, 0, s>>>(x, y, wc, w.ranks, tm, d, N);
    else
      k_toep_last<T, T, 0, 1><<<gl, 256, 0, s>>>(x, y, wc, w.ranks, tm, d, N);
    QTT_LAUNCH_CHECK();
    return QTT_OK;
  }
  const double* cur = nullptr;
  for (int k = 1; k < d; ++k) {
    double* nxt = buf[(k - 1) & 1];
    const int gy = (2 * w.cap[k] + 4 * kToepNB - 1) / (4 * kToepNB);
    dim3 grid((unsigned)((half + 63) / 64), (unsigned)gy);
    if (k == 1) {
      if (trans)
        k_toep_step<T, T, 1, 1><<<grid, 256, 0, s>>>(x, nxt, wc, w.ranks, tm, k, N);
      else
        k_toep_step<T, T, 0, 1><<<grid, 256, 0, s>>>(x, nxt, wc, w.ranks, tm, k, N);
    } else {
      if (trans)
        k_toep_step<T, double, 1, 0><<<grid, 256, 0, s>>>(cur, nxt, wc, w.ranks, tm, k, N);
      else
        k_toep_step<T, double, 0, 0><<<grid, 256, 0, s>>>(cur, nxt, wc, w.ranks, tm, k, N);
    }
    QTT_LAUNCH_CHECK();
    cur = nxt;
  }
  if (trans)
    k_toep_last<T, double, 1, 0><<<gl, 256, 0, s>>>(cur, y, wc, w.ranks, tm, d, N);
  else
    k_toep_last<T, double, 0, 0><<<gl, 256, 0, s>>>(cur, y, wc, w.ranks, tm, d, N);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_toeplitz(const TensorDev& w, int dtype, const void* x, void* y, int trans, void* ws,
                 hipStream_t s) {
  if (dtype == QTT_F64)
    return toeplitz_t<double>(w, static_cast<const double*>(x), static_cast<double*>(y), trans,
                              static_cast<double*>(ws), s);
  return toeplitz_t<float>(w, static_cast<const float*>(x), static_cast<float*>(y), trans,
                           static_cast<double*>(ws), s);
}

__global__ void k_copy_ranks(const int32_t* src, int32_t* dst, int n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// ================================================ kernel-core gradients
// For L with upstream gradient g = dL/dy of y = T(w) f, the gradient with
// respect to core k of the generator (k = 1..d+1) contracts the transposed
// product's state before mode k with the forward product's state after it:
//   P_{k-1}[(a,c)][pos]: g pushed through modes 1..k-1 of T^T (bits < k of
//     pos are i, bits >= k are j; P_0 = g with a = 0 and carry-in 1);
//   Q_k[(b,c')][pos]: f pushed through modes k+1..d of T from the top, the
//     top bit u_{d+1} = c_d contracted with W_{d+1} (bits <= k of pos are i,
//     bits > k are j; Q_d = W_{d+1}[b, c', 0] f);
//   dL/dW_k[a, u, b] = sum_{pos'} sum_{o, n, c} P_{k-1}[(a,c)][pos'|o]
//       Q_k[(b,c')][pos'|n] [u = (o + 1 - n + c) mod 2, c' = (o + 1 - n + c) div 2]
// where pos' runs over the positions without bit k, o = j_k and n = i_k.
// Core d+1 (u = c_d): dL/dW_{d+1}[a, c, 0] = sum_pos P_d[(a,c)][pos] f[pos].
// The Q states are computed top-down and kept (the P states run bottom-up);
// every sum is FP64 in a fixed order.

// Q_d = W_{d+1}[b, c', 0] f, b2 = 2 b + c' < 2 rho_d
template <typename T>
__global__ void __launch_bounds__(256) k_toep_qfirst(const T* f, double* out, const T* wc,
                                                     const int32_t* wr, ToepMeta tm, int d,
                                                     long long N) {
  const long long pos = (long long)blockIdx.x * 256 + threadIdx.x;
  if (pos >= N) return;
  const int nb = 2 * wr[d];
  const T* Wl = wc + tm.woff[d];  // (rho_d, 2, 1): entry b2 = 2 b + c'
  const double fv = (double)f[pos];
  for (int b2 = 0; b2 < nb; ++b2) out[(long long)b2 * N + pos] = (double)Wl[b2] * fv;
}

// Q_{k-1} from Q_k: Q_{k-1}[(a,c)][..o..] = sum_{n,b} W_k[a, u, b] Q_k[(b,c')][..n..]
// (bit k-1 of pos, 0-based: o on the output, n on the input)
template <typename T>
__global__ void __launch_bounds__(256) k_toep_qstep(const double* in, double* out, const T* wc,
                                                    const int32_t* wr, ToepMeta tm, int k,
                                                    long long N) {
  const long long half = N >> 1;
  const long long q = (long long)blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  const int rin = wr[k];       // bond of Q_k (right rank of W_k)
  const int rout = wr[k - 1];  // bond of Q_{k-1} (left rank of W_k)
  const int b0 = (blockIdx.y * 4 + w) * kToepNB;  // first output bond of this thread
  if (b0 >= 2 * rout || q >= half) return;
  const T* Wk = wc + tm.woff[k - 1];  // W_k[a][u][b] at (a*2 + u)*rin + b
  const int bit = k - 1;
  const long long p0 = ins_bit(q, bit, 0), p1 = ins_bit(q, bit, 1);
  double acc[kToepNB][2];
#pragma unroll
  for (int t = 0; t < kToepNB; ++t) acc[t][0] = acc[t][1] = 0.0;
  for (int b = 0; b < rin; ++b) {
#pragma unroll
    for (int c1 = 0; c1 < 2; ++c1) {
      const long long row = (long long)(2 * b + c1) * N;
      const double x0 = in[row + p0], x1 = in[row + p1];
#pragma unroll
      for (int t = 0; t < kToepNB; ++t) {
        const int bo = b0 + t;
        if (bo < 2 * rout) {
          const int a = bo >> 1, c = bo & 1;
#pragma unroll
          for (int o = 0; o < 2; ++o) {
#pragma unroll
            for (int n = 0; n < 2; ++n) {
              const int v = o + (1 - n) + c;
              if ((v >> 1) == c1) {
                const double wv = (double)Wk[(a * 2 + (v & 1)) * rin + b];
                acc[t][o] = fma(wv, n ? x1 : x0, acc[t][o]);
              }
            }
          }
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kToepNB; ++t) {
    const int bo = b0 + t;
    if (bo < 2 * rout) {
      out[(long long)bo * N + p0] = acc[t][0];
      out[(long long)bo * N + p1] = acc[t][1];
    }
  }
}

constexpr int kWgChunk = 16;   // positions pos' staged per pass
constexpr int kWgBlocks = 256; // partial sums per core

// partial dL/dW_k (k = 1..d) over chunks of pos': part[blk][(a*2 + u)*rb + b].
// P is the transposed product's state P_{k-1} (FP64), or g itself when FIRST.
template <typename T, int FIRST>
__global__ void __launch_bounds__(256) k_wgrad_part(const void* pin, const double* qin,
                                                    const int32_t* wr, int k, long long N,
                                                    double* part, int max_out) {
  extern __shared__ double wg_lds[];
  const int ra = FIRST ? 1 : wr[k - 1], rb = wr[k];
  const int npa = 2 * ra, npb = 2 * rb;
  // Ps[(2a + c)][o][cc], Qs[(2b + c')][n][cc]
  double* Ps = wg_lds;
  double* Qs = wg_lds + (size_t)npa * 2 * kWgChunk;
  const int nout = ra * 2 * rb;
  const int tid = threadIdx.x;
  const long long half = N >> 1;
  const int bit = k - 1;
  double acc[32];
#pragma unroll
  for (int t = 0; t < 32; ++t) acc[t] = 0.0;
  const long long nch = (half + kWgChunk - 1) / kWgChunk;
  for (long long ch = blockIdx.x; ch < nch; ch += gridDim.x) {
    const long long base = ch * kWgChunk;
    for (int e = tid; e < npa * 2 * kWgChunk; e += 256) {
      const int row = e / (2 * kWgChunk), rem = e - row * (2 * kWgChunk);
      const int o = rem / kWgChunk, cc = rem - o * kWgChunk;
      const long long qq = base + cc;
      double v = 0.0;
      if (qq < half) {
        const long long p = ins_bit(qq, bit, o);
        if (FIRST)
          v = (row == 1) ? (double)static_cast<const T*>(pin)[p] : 0.0;  // a = 0, carry-in 1
        else
          v = static_cast<const double*>(pin)[(long long)row * N + p];
      }
      Ps[e] = v;
    }
    for (int e = tid; e < npb * 2 * kWgChunk; e += 256) {
      const int row = e / (2 * kWgChunk), rem = e - row * (2 * kWgChunk);
      const int n = rem / kWgChunk, cc = rem - n * kWgChunk;
      const long long qq = base + cc;
      Qs[e] = qq < half ? qin[(long long)row * N + ins_bit(qq, bit, n)] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int oi = tid + 256 * t;
      if (oi < nout) {
        const int a = oi / (2 * rb), rem = oi - a * 2 * rb;
        const int u = rem / rb, b = rem - u * rb;
        double s = acc[t];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int n = (o + 1 + c + u) & 1;
            const int c1 = (o + 1 - n + c) >> 1;
            const double* pp = Ps + ((2 * a + c) * 2 + o) * kWgChunk;
            const double* qp = Qs + ((2 * b + c1) * 2 + n) * kWgChunk;
#pragma unroll
            for (int cc = 0; cc < kWgChunk; ++cc) s = fma(pp[cc], qp[cc], s);
          }
        }
        acc[t] = s;
      }
    }
    __syncthreads();
  }
  double* P = part + (size_t)blockIdx.x * max_out;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int oi = tid + 256 * t;
    if (oi < nout) P[oi] = acc[t];
  }
}

// partial dL/dW_{d+1}[a, c, 0] = sum_pos P_d[(a,c)][pos] f[pos]: block (x, b2)
template <typename T>
__global__ void __launch_bounds__(256) k_wgrad_top_part(const double* pd, const T* f,
                                                        long long N, double* part,
                                                        int max_out) {
  __shared__ double red[256];
  const int b2 = blockIdx.y;
  double s = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < N;
       e += (long long)gridDim.x * 256)
    s = fma(pd[(long long)b2 * N + e], (double)f[e], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)blockIdx.x * max_out + b2] = red[0];
}

template <typename T>
__global__ void k_wgcore_sum(const double* part, int nblk, int max_out, const int32_t* ranks,
                             int k, T* gcores, long long off) {
  const int nout = 2 * ranks[k - 1] * ranks[k];
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * max_out + o];
  gcores[off + o] = (T)s;
}

struct WgPlan {
  long long qoff[QTT_MAXD + 2];  // element offset of the stored Q_k (k = 1..d)
  size_t q_elems;
  size_t p_elems;                // one P buffer: 2 max_{k=1..d} cap_k N
  int max_out;                   // max_k 2 cap_{k-1} cap_k over the d+1 cores
};

static void wg_plan(int d, const int32_t* wcap, WgPlan* p) {
  const long long N = 1LL << d;
  long long o = 0;
  int rmax = 1, mo = 1;
  for (int k = 1; k <= d; ++k) {
    p->qoff[k] = o;
    o += 2LL * wcap[k] * N;
    if (wcap[k] > rmax) rmax = wcap[k];
  }
  for (int k = 1; k <= d + 1; ++k) {
    const int oc = 2 * wcap[k - 1] * wcap[k];
    if (oc > mo) mo = oc;
  }
  p->q_elems = (size_t)o;
  p->p_elems = (size_t)(2 * rmax) * (size_t)N;
  p->max_out = mo;
}

size_t wgrad_ws_bytes(int d, const int32_t* w_cap) {
  WgPlan p;
  wg_plan(d, w_cap, &p);
  Arena ar(nullptr);
  ar.take<double>(p.q_elems);
  ar.take<double>(p.p_elems);
  ar.take<double>(p.p_elems);
  ar.take<double>((size_t)kWgBlocks * p.max_out);
  return ar.size();
}

static size_t wgrad_lds(int ra_cap, int rb_cap) {
  return (size_t)(2 * ra_cap + 2 * rb_cap) * 2 * kWgChunk * sizeof(double);
}

template <typename T>
static int conv_backward_w_t(const TensorDev& w, const T* f, const T* gy, T* gf,
                             const TensorDev& gw, void* ws, hipStream_t s) {
  const int d = w.d - 1;
  const long long N = 1LL << d, half = N >> 1;
  WgPlan p;
  wg_plan(d, w.cap, &p);
  Arena ar(ws);
  double* qs = ar.take<double>(p.q_elems);
  double* pb[2] = {ar.take<double>(p.p_elems), ar.take<double>(p.p_elems)};
  double* part = ar.take<double>((size_t)kWgBlocks * p.max_out);
  ToepMeta tm;
  for (int k = 0; k <= w.d; ++k) tm.woff[k] = w.off[k];
  const T* wc = static_cast<const T*>(w.cores);
  T* G = static_cast<T*>(gw.cores);
  for (int k = 1; k <= d; ++k) {
    const size_t lds = wgrad_lds(k == 1 ? 1 : w.cap[k - 1], w.cap[k]);
    if (lds > 64 * 1024) return QTT_ENOTSUP;
  }
  static std::once_flag attr_once;
  static hipError_t attr_err = hipSuccess;
  std::call_once(attr_once, [] {
    const int mx = (int)wgrad_lds(kMaxRank, kMaxRank);
    set_lds_limit((const void*)k_wgrad_part<T, 0>, mx, &attr_err);
    set_lds_limit((const void*)k_wgrad_part<T, 1>, mx, &attr_err);
  });
  QTT_HIP_CHECK(attr_err);
  ProbeScope _ps(QTT_K_ADJOINT, s);
  k_copy_ranks<<<1, 64, 0, s>>>(w.ranks, gw.ranks, d + 2);
  QTT_LAUNCH_CHECK();
  // Q_d .. Q_1, top-down, all kept
  k_toep_qfirst<T><<<(unsigned)((N + 255) / 256), 256, 0, s>>>(f, qs + p.qoff[d], wc, w.ranks, tm,
                                                               d, N);
  QTT_LAUNCH_CHECK();
  for (int k = d; k >= 2; --k) {
    const int gyd = (2 * w.cap[k - 1] + 4 * kToepNB - 1) / (4 * kToepNB);
    dim3 grid((unsigned)((half + 63) / 64), (unsigned)gyd);
    k_toep_qstep<T><<<grid, 256, 0, s>>>(qs + p.qoff[k], qs + p.qoff[k - 1], wc, w.ranks, tm, k,
                                        N);
    QTT_LAUNCH_CHECK();
  }
  // P sweep bottom-up with the gradient of core k from P_{k-1} and Q_k
  const long long nch = (half + kWgChunk - 1) / kWgChunk;
  const int nblk = (int)(nch < kWgBlocks ? nch : kWgBlocks);
  const double* pcur = nullptr;
  for (int k = 1; k <= d; ++k) {
    const size_t lds = wgrad_lds(k == 1 ? 1 : w.cap[k - 1], w.cap[k]);
    if (k == 1)
      k_wgrad_part<T, 1><<<nblk, 256, lds, s>>>(gy, qs + p.qoff[k], w.ranks, k, N, part,
                                                p.max_out);
    else
      k_wgrad_part<T, 0><<<nblk, 256, lds, s>>>(pcur, qs + p.qoff[k], w.ranks, k, N, part,
                                                p.max_out);
    QTT_LAUNCH_CHECK();
    const int nout = 2 * w.cap[k - 1] * w.cap[k];
    k_wgcore_sum<T><<<(nout + 255) / 256, 256, 0, s>>>(part, nblk, p.max_out, w.ranks, k, G,
                                                       gw.off[k - 1]);
    QTT_LAUNCH_CHECK();
    // P_k (k = d included: the top core's gradient needs P_d)
    double* nxt = pb[(k - 1) & 1];
    const int gyd = (2 * w.cap[k] + 4 * kToepNB - 1) / (4 * kToepNB);
    dim3 grid((unsigned)((half + 63) / 64), (unsigned)gyd);
    if (k == 1)
      k_toep_step<T, T, 1, 1><<<grid, 256, 0, s>>>(gy, nxt, wc, w.ranks, tm, k, N);
    else
      k_toep_step<T, double, 1, 0><<<grid, 256, 0, s>>>(pcur, nxt, wc, w.ranks, tm, k, N);
    QTT_LAUNCH_CHECK();
    if (k == d) {
      // the transposed product itself from P_{d-1} (or g when d = 1)
      const unsigned gl = (unsigned)((half + 255) / 256);
      if (d == 1)
        k_toep_last<T, T, 1, 1><<<gl, 256, 0, s>>>(gy, gf, wc, w.ranks, tm, d, N);
      else
        k_toep_last<T, double, 1, 0><<<gl, 256, 0, s>>>(pcur, gf, wc, w.ranks, tm, d, N);
      QTT_LAUNCH_CHECK();
    }
    pcur = nxt;
  }
  // core d+1 from P_d and f
  {
    const int nb2 = 2 * w.cap[d];
    long long nbx = (N + 255) / 256;
    if (nbx > kWgBlocks) nbx = kWgBlocks;
    dim3 grid((unsigned)nbx, (unsigned)nb2);
    k_wgrad_top_part<T><<<grid, 256, 0, s>>>(pcur, f, N, part, p.max_out);
    QTT_LAUNCH_CHECK();
    k_wgcore_sum<T><<<(nb2 + 255) / 256, 256, 0, s>>>(part, (int)nbx, p.max_out, w.ranks, d + 1,
                                                      G, gw.off[d]);
    QTT_LAUNCH_CHECK();
  }
  return QTT_OK;
}

int run_conv_backward_w(const TensorDev& w, int dtype, const void* f, const void* gy, void* gf,
                        const TensorDev& gw, void* ws, hipStream_t s) {
  if (dtype == QTT_F64)
    return conv_backward_w_t<double>(w, static_cast<const double*>(f),
                                     static_cast<const double*>(gy), static_cast<double*>(gf), gw,
                                     ws, s);
  return conv_backward_w_t<float>(w, static_cast<const float*>(f), static_cast<const float*>(gy),
                                  static_cast<float*>(gf), gw, ws, s);
}

// ========================================================== full adjoint
// For G = <g, full(F)>:  dG/dF_k[a, i, b] = sum_rest H_{k-1}[a][i + 2 rest] Rf_k[b][rest]
// with the right interfaces Rf_k (r_k x 2^(d-k)),
//   Rf_d = 1,  Rf_{k-1}[a][i + 2 rest] = sum_b F_k[a, i, b] Rf_k[b][rest],
// and the left partial contractions H_k (r_k x 2^(d-k)),
//   H_0 = g,  H_k[b][rest] = sum_{a,i} F_k[a, i, b] H_{k-1}[a][i + 2 rest].
struct AdjPlan {
  long long rfoff[QTT_MAXD + 1];  // element offset of Rf_k (k = 1..d)
  size_t rf_elems;
  size_t h_elems;                 // one H buffer
  int max_out;                    // max 2 cap_{k-1} cap_k
};

static void adj_plan(int d, const int* cap, AdjPlan* p) {
  long long o = 0;
  size_t hmax = 1;
  int mo = 1;
  for (int k = 1; k <= d; ++k) {
    p->rfoff[k] = o;
    const long long e = (long long)cap[k] << (d - k);
    o += e;
    if ((size_t)e > hmax) hmax = (size_t)e;
    const int oc = 2 * cap[k - 1] * cap[k];
    if (oc > mo) mo = oc;
  }
  p->rf_elems = (size_t)o;
  p->h_elems = hmax;
  p->max_out = mo;
}

template <typename T>
__global__ void k_rf_one(T* rf) {
  if (threadIdx.x == 0) rf[0] = (T)1;
}

// Rf_{k-1} from Rf_k: thread per (a, col), col = i + 2 rest < 2M, M = 2^(d-k)
template <typename T>
__global__ void __launch_bounds__(256) k_rf_step(const T* Fk, const int32_t* ranks, int k,
                                                 const T* rfk, T* rfk1, long long M) {
  const int r0 = ranks[k - 1], r1 = ranks[k];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long cols = 2 * M;
  const int a = (int)(e / cols);
  if (a >= r0) return;
  const long long col = e - (long long)a * cols;
  const int i = (int)(col & 1);
  const long long rest = col >> 1;
  double s = 0.0;
  for (int b = 0; b < r1; ++b)
    s = fma((double)Fk[(a * 2 + i) * r1 + b], (double)rfk[(long long)b * M + rest], s);
  rfk1[(long long)a * cols + col] = (T)s;
}

// H_k from H_{k-1}: thread per (b, rest), rest < M = 2^(d-k)
template <typename T>
__global__ void __launch_bounds__(256) k_h_step(const T* Fk, const int32_t* ranks, int k,
                                                const T* hin, T* hout, long long M) {
  const int r0 = ranks[k - 1], r1 = ranks[k];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int b = (int)(e / M);
  if (b >= r1) return;
  const long long rest = e - (long long)b * M;
  double s = 0.0;
  for (int a = 0; a < r0; ++a) {
    const T* h = hin + (long long)a * 2 * M + 2 * rest;
    s = fma((double)Fk[(a * 2) * r1 + b], (double)h[0], s);
    s = fma((double)Fk[(a * 2 + 1) * r1 + b], (double)h[1], s);
  }
  hout[(long long)b * M + rest] = (T)s;
}

constexpr int kGcChunk = 32;
constexpr int kGcBlocks = 256;

// partial core gradients over chunks of rest: part[blk][(a*2+i)*r1 + b]
template <typename T>
__global__ void __launch_bounds__(256) k_gcore_part(const T* hprev, const T* rfk,
                                                    const int32_t* ranks, int k, long long M,
                                                    double* part, int max_out) {
  __shared__ double Hs[2 * kMaxRank][kGcChunk + 1];
  __shared__ double Rs[kMaxRank][kGcChunk + 1];
  const int r0 = ranks[k - 1], r1 = ranks[k];
  const int nout = 2 * r0 * r1;
  const int tid = threadIdx.x;
  double acc[32];
#pragma unroll
  for (int t = 0; t < 32; ++t) acc[t] = 0.0;
  const long long nchunks = (M + kGcChunk - 1) / kGcChunk;
  for (long long ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const long long base = ch * kGcChunk;
    for (int e = tid; e < 2 * r0 * kGcChunk; e += 256) {
      const int row = e / kGcChunk, cc = e - row * kGcChunk;  // row = a*2 + i
      const long long rest = base + cc;
      const int a = row >> 1, i = row & 1;
      Hs[row][cc] = rest < M ? (double)hprev[(long long)a * 2 * M + i + 2 * rest] : 0.0;
    }
    for (int e = tid; e < r1 * kGcChunk; e += 256) {
      const int b = e / kGcChunk, cc = e - b * kGcChunk;
      const long long rest = base + cc;
      Rs[b][cc] = rest < M ? (double)rfk[(long long)b * M + rest] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int o = tid + 256 * t;
      if (o < nout) {
        const int row = o / r1, b = o - row * r1;
        double s = acc[t];
        for (int cc = 0; cc < kGcChunk; ++cc) s = fma(Hs[row][cc], Rs[b][cc], s);
        acc[t] = s;
      }
    }
    __syncthreads();
  }
  double* P = part + (size_t)blockIdx.x * max_out;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int o = tid + 256 * t;
    if (o < nout) P[o] = acc[t];
  }
}

// fixed-order sum of the partials into core k of the gradient tensor
template <typename T>
__global__ void k_gcore_sum(const double* part, int nblk, int max_out, const int32_t* ranks,
                            int k, T* gcores, long long off) {
  const int nout = 2 * ranks[k - 1] * ranks[k];
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(size_t)b * max_out + o];
  gcores[off + o] = (T)s;
}

size_t full_adjoint_ws_bytes(int d, const int* cap, int dtype) {
  AdjPlan p;
  adj_plan(d, cap, &p);
  const size_t es = elem_size(dtype);
  Arena ar(nullptr);
  ar.take<char>(p.rf_elems * es);
  ar.take<char>(p.h_elems * es);
  ar.take<char>(p.h_elems * es);
  ar.take<double>((size_t)kGcBlocks * p.max_out);
  return ar.size();
}

template <typename T>
static int full_adjoint_t(const TensorDev& f, const T* g, const TensorDev& gr, void* ws,
                          hipStream_t s) {
  const int d = f.d;
  AdjPlan p;
  adj_plan(d, f.cap, &p);
  Arena ar(ws);
  T* rf = ar.take<T>(p.rf_elems);
  T* hb[2] = {ar.take<T>(p.h_elems), ar.take<T>(p.h_elems)};
  double* part = ar.take<double>((size_t)kGcBlocks * p.max_out);
  const T* F = static_cast<const T*>(f.cores);
  T* G = static_cast<T*>(gr.cores);
  ProbeScope _ps(QTT_K_ADJOINT, s);
  k_copy_ranks<<<1, 64, 0, s>>>(f.ranks, gr.ranks, d + 1);
  QTT_LAUNCH_CHECK();
  // right interfaces Rf_d .. Rf_1
  k_rf_one<T><<<1, 64, 0, s>>>(rf + p.rfoff[d]);
  QTT_LAUNCH_CHECK();
  for (int k = d; k >= 2; --k) {
    const long long M = 1LL << (d - k);
    const long long total = (long long)f.cap[k - 1] * 2 * M;
    const unsigned gx = (unsigned)((total + 255) / 256);
    k_rf_step<T><<<gx, 256, 0, s>>>(F + f.off[k - 1], f.ranks, k, rf + p.rfoff[k],
                                    rf + p.rfoff[k - 1], M);
    QTT_LAUNCH_CHECK();
  }
  // left sweep: gradient of core k from H_{k-1} and Rf_k, then H_k
  const T* hprev = g;
  for (int k = 1; k <= d; ++k) {
    const long long M = 1LL << (d - k);
    const long long nch = (M + kGcChunk - 1) / kGcChunk;
    const int nblk = (int)(nch < kGcBlocks ? nch : kGcBlocks);
    k_gcore_part<T><<<nblk, 256, 0, s>>>(hprev, rf + p.rfoff[k], f.ranks, k, M, part, p.max_out);
    QTT_LAUNCH_CHECK();
    const int nout = 2 * f.cap[k - 1] * f.cap[k];
    k_gcore_sum<T><<<(nout + 255) / 256, 256, 0, s>>>(part, nblk, p.max_out, f.ranks, k, G,
                                                      gr.off[k - 1]);
    QTT_LAUNCH_CHECK();
    if (k < d) {
      T* hn = hb[(k - 1) & 1];
      const long long total = (long long)f.cap[k] * M;
      k_h_step<T><<<(unsigned)((total + 255) / 256), 256, 0, s>>>(F + f.off[k - 1], f.ranks, k,
                                                                   hprev, hn, M);
      QTT_LAUNCH_CHECK();
      hprev = hn;
    }
  }
  return QTT_OK;
}

int run_full_adjoint(const TensorDev& f, int dtype, const void* g, const TensorDev& gr, void* ws,
                     hipStream_t s) {
  if (dtype == QTT_F64)
    return full_adjoint_t<double>(f, static_cast<const double*>(g), gr, ws, s);
  return full_adjoint_t<float>(f, static_cast<const float*>(g), gr, ws, s);
}

// ================================================================== dot
constexpr int kDotBlocks = kDotPartials;

template <typename T>
__global__ void __launch_bounds__(256) k_dot_part(const T* a, const T* b, long long n,
                                                  double* part) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n;
       e += (long long)gridDim.x * 256)
    s = fma((double)a[e], (double)b[e], s);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// *out = sum of the block partials, in block order
__global__ void k_dot_final(const double* part, int nblk, double* out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[b];
    *out = s;
  }
}

template <typename T>
static int dot_t(const T* a, const T* b, long long n, double* part, double* out, hipStream_t s) {
  long long nb = (n + 255) / 256;
  if (nb > kDotBlocks) nb = kDotBlocks;
  if (nb < 1) nb = 1;
  k_dot_part<T><<<(unsigned)nb, 256, 0, s>>>(a, b, n, part);
  QTT_LAUNCH_CHECK();
  k_dot_final<<<1, 64, 0, s>>>(part, (int)nb, out);
  QTT_LAUNCH_CHECK();
  return QTT_OK;
}

int run_dot(int dtype, const void* a, const void* b, long long n, double* part, double* out,
            hipStream_t s) {
  if (dtype == QTT_F64)
    return dot_t<double>(static_cast<const double*>(a), static_cast<const double*>(b), n, part,
                         out, s);
  return dot_t<float>(static_cast<const float*>(a), static_cast<const float*>(b), n, part, out, s);
}

// ================================================= sinc derivative sums
// c[0] = 1/S, c[1] = S'/S with S = sum_m s_m, S' = sum_m ds_m/dB over the
// 2^nk kernel samples (fixed-order block sums).
__global__ void __launch_bounds__(256) k_sinc_sums(double B, int nk, double* part) {
  __shared__ double r0[256], r1[256];
  const long long nn = 1LL << nk;
  double s0 = 0.0, s1 = 0.0;
  for (long long m = (long long)blockIdx.x * 256 + threadIdx.x; m < nn;
       m += (long long)gridDim.x * 256) {
    double sv, dv;
    sinc_gen_pair(m + (nn >> 1), B, nk, &sv, &dv);
    s0 += sv;
    s1 += dv;
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r0[threadIdx.x] += r0[threadIdx.x + h];
      r1[threadIdx.x] += r1[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r0[0];
    part[2 * blockIdx.x + 1] = r1[0];
  }
}

__global__ void k_sinc_sums_final(const double* part, int nblk, double* c) {
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int b = 0; b < nblk; ++b) {
      s0 += part[2 * b];
      s1 += part[2 * b + 1];
    }
    c[0] = s0 != 0.0 ? 1.0 / s0 : 0.0;
    c[1] = s0 != 0.0 ? s1 / s0 : 0.0;
  }
}

constexpr int kSumBlocks = 256;

size_t sinc_sums_ws_bytes() {
  Arena ar(nullptr);
  ar.take<double>(2);
  ar.take<double>(2 * kSumBlocks);
  return ar.size();  // a multiple of 256
}

int run_sinc_sums(double B, int nk, void* ws, double** consts, hipStream_t s) {
  Arena ar(ws);
  double* c = ar.take<double>(2);
  double* part = ar.take<double>(2 * kSumBlocks);
  const long long nn = 1LL << nk;
  long long nb = (nn + 255) / 256;
  if (nb > kSumBlocks) nb = kSumBlocks;
  ProbeScope _ps(QTT_K_OTHER, s);
  k_sinc_sums<<<(unsigned)nb, 256, 0, s>>>(B, nk, part);
  QTT_LAUNCH_CHECK();
  k_sinc_sums_final<<<1, 64, 0, s>>>(part, (int)nb, c);
  QTT_LAUNCH_CHECK();
  *consts = c;
  return QTT_OK;
}

}  // namespace qtt

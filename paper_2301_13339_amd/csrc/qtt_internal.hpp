// Internal declarations shared by the HIP translation units of libqtt.
//
// Constants, the launch probe, the decomposition plan and a small host arena
// that carves the caller's workspace.  Every truncated SVD goes through the
// Gram matrix of the unfolding and the one-workgroup FP64 symmetric
// eigensolver of qtt_syev.hpp; the truncation rule of Algorithm 1 with the
// max-rank modification (1) is in qtt_eig.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "qtt.h"

namespace qtt {

// ----------------------------------------------------------------- limits
constexpr int kMaxRank = QTT_MAX_RANK;       // largest TT-rank of a decomposition
constexpr int kMaxM = 2 * kMaxRank;          // largest unfolding row count m_k = 2 r_{k-1}
constexpr int kLevel = 6;                    // levels handled from one data Gram (2^6 = 64)
constexpr int kTailElems = 8192;             // remainder size a single workgroup finishes in LDS
constexpr int kEigLds = 64;                  // eigen problems up to this size live in LDS
constexpr int kMaxPartials = 128;            // partial Gram matrices per streaming pass
constexpr int kSvStride = 2 * kMaxRank;      // row stride of the optional singular-value output

// ------------------------------------------------------------ LDS pointers
// A plain pointer argument of a device function that is not inlined is a
// generic address, and every access through it is a flat instruction (the
// latency of a global access and a wait on both memory counters) even when
// it points into LDS.  The eigensolver passes its LDS arrays as pointers in
// address space 3 instead, so that they compile to ds_* instructions.
template <class T>
using lds_ptr = __attribute__((address_space(3))) T*;
using ldsd = lds_ptr<double>;
using ldsi = lds_ptr<int>;
template <class T>
__device__ __forceinline__ lds_ptr<T> lds(T* p) {
  return (lds_ptr<T>)p;
}

// -------------------------------------------------------------- host arena
struct Arena {
  char* base;
  size_t off;
  explicit Arena(void* b) : base(static_cast<char*>(b)), off(0) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += n * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~size_t(255); }
};

inline size_t elem_size(int dtype) { return dtype == QTT_F64 ? 8 : 4; }

// offsets (elements) of the cores for capacities cap[0..d]
inline size_t core_offset(const int32_t* cap, int k) {  // k is 0-based core index
  size_t off = 0;
  for (int j = 0; j < k; ++j) off += size_t(cap[j]) * 2 * size_t(cap[j + 1]);
  return off;
}

// Device-side description of a QTT tensor: capacities are baked into the
// per-core offsets; actual ranks are read from device memory.
struct TensorDev {
  int d;
  int32_t* ranks;
  void* cores;
  int32_t* status;
  long long off[QTT_MAXD + 1];  // element offsets of cores 0..d-1 (off[d] = total)
  int cap[QTT_MAXD + 1];
};

inline TensorDev make_dev(const qtt_tensor* t) {
  TensorDev o;
  o.d = t->d;
  o.ranks = t->ranks;
  o.cores = t->cores;
  o.status = t->status;
  long long off = 0;
  for (int k = 0; k <= t->d; ++k) {
    o.cap[k] = t->cap[k];
    o.off[k] = off;
    if (k < t->d) off += (long long)t->cap[k] * 2 * t->cap[k + 1];
  }
  return o;
}

// ------------------------------------------------------------ launch probe
// Records a HIP event pair around launches of the probed class (see
// qtt_probe_start).  Cheap no-op when the class is not probed.
void probe_pre(int cls, hipStream_t s);
void probe_post(int cls, hipStream_t s);
struct ProbeScope {
  int cls;
  hipStream_t s;
  ProbeScope(int c, hipStream_t st) : cls(c), s(st) { probe_pre(c, st); }
  ~ProbeScope() { probe_post(cls, s); }
};

// ------------------------------------------------------------ host errors
void set_hip_error(hipError_t e);
#define QTT_HIP_CHECK(expr)                     \
  do {                                          \
    hipError_t _e = (expr);                     \
    if (_e != hipSuccess) {                     \
      ::qtt::set_hip_error(_e);                 \
      return QTT_EHIP;                          \
    }                                           \
  } while (0)
// Raise the dynamic-LDS limit of a kernel; keeps the first failure in *err.
inline void set_lds_limit(const void* fn, int bytes, hipError_t* err) {
  const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess && *err == hipSuccess) *err = e;
}
#define QTT_LAUNCH_CHECK()                      \
  do {                                          \
    hipError_t _e = hipGetLastError();          \
    if (_e != hipSuccess) {                     \
      ::qtt::set_hip_error(_e);                 \
      return QTT_EHIP;                          \
    }                                           \
  } while (0)

// ------------------------------------------------------- decomposition API
// Sample source for the decomposition sweep: a stored vector, or the sinc
// generator evaluated on the fly.
struct Source {
  const void* x;     // stored samples (nullptr when generated)
  int gen;           // 1: sinc generator of a 2^(D-1)-sample kernel grid
  double B;          // generator bandwidth
  int nk;            // generator: log2 of the kernel grid size (D - 1)
};

struct DecompPlan {
  int D;             // modes
  int dtype;
  int rcap;          // effective rank cap
  int cap[QTT_MAXD + 1];
  int use_level;     // 1 when the level start is used
  int tail_k;        // first step handled by the tail kernel (1-based)
  // workspace pieces
  double* scal;      // [0]=||x||^2, [1]=tau^2, [2]=generator sum, [3..] reserved
  int32_t* iflags;   // [0] non-finite flag
  double* partials;  // kMaxPartials * pstride
  double* gram;      // reduced Gram, gstride*gstride
  double* umat;      // projection matrix (rows x r)
  double* eigA;      // global scratch for eigen problems larger than kEigLds
  double* eigV;
  void* xbuf[2];     // remainder buffers (elements of dtype)
  double* gpart_sum; // partial sums of generator samples
  size_t ws_bytes;
  int pstride;       // doubles per partial Gram
  int gstride;       // row stride of the reduced Gram
};

int plan_decompose(int D, int rcap, int dtype, void* ws, DecompPlan* p);
// delta: drop-off threshold of modification (3) of Section 5 (0 = off)
int run_decompose(const DecompPlan& p, const Source& src, double eps, const TensorDev& out,
                  double* sv, hipStream_t stream, double delta = 0.0);

// ----------------------------------------------------------------- batched
// One independent decomposition of a batch (see k_batch_decompose).
struct BatchTask {
  long long x_off;     // offset of the samples (stored samples only)
  long long core_off;  // element offset of the task's cores (capacity strided)
  int rank_off;        // offset of its D+1 ranks
  int status_idx;      // its status word
  int D;               // binary modes
  int rcap;            // rank capacity, 1..kMaxRank
  int nk;              // generator: log2 of the kernel grid
  int pad;
  double B;            // generator bandwidth
  double eps;          // tolerance
};

// doubles of per-workgroup scratch ahead of the two remainder buffers
constexpr long long batch_wg_doubles() {
  return 16 + (long long)kMaxM * kMaxRank + 2LL * (kMaxM + 1) * (kMaxM + 1);
}

int run_batch_decompose(int dtype, int gen, const void* x, const BatchTask* tasks, int ntasks,
                        int32_t* counter, void* cores, int32_t* ranks, int32_t* status,
                        char* wscr, long long wstride, long long nmax, int nwg, hipStream_t s);
size_t batch_decompose_lds();

int launch_reduce(const double* partials, int pstride, int nparts, int count, double* out,
                  hipStream_t s);

// ------------------------------------------------------ general mode sizes
// TT-SVD / max-rank TT-RSVD of a tensor with K modes of size M (FP64)
constexpr int kModesMaxM = 64;    // largest mode size
int modes_caps(int K, int M, int max_rank, int32_t* cap);
size_t modes_ws_bytes(int K, int M, int method, int oversample);
int run_decompose_modes(const double* x, int K, int M, double eps, int method, int oversample,
                        uint64_t seed, const int32_t* cap, int32_t* ranks, double* cores,
                        int32_t* status, int lib_capped, void* ws, hipStream_t s);

// --------------------------------------------------------------- other ops
int plan_full(int d, const int32_t* cap, int dtype, void* ws, size_t* ws_bytes, void** bufs);
int run_full(const TensorDev& t, int dtype, void* out, void* ws, hipStream_t stream);

int run_conv(const TensorDev& f, const TensorDev* w, int n_axes, const int32_t* axis_modes,
             const TensorDev& y, int dtype, hipStream_t stream);

// ------------------------------------------------------------------- sketch
size_t sketch_ws_bytes(int D, int dtype, int ell);
int run_round_sketch(int dtype, int bf16, const void* y, int D, double eps, const int* cap,
                     int ell, uint64_t seed, const TensorDev& out, void* ws, hipStream_t s);

// ------------------------------------------------------------------ adjoint
size_t toeplitz_ws_elems(int d, const int32_t* w_cap);
int run_toeplitz(const TensorDev& w, int dtype, const void* x, void* y, int trans, void* ws,
                 hipStream_t s);
size_t full_adjoint_ws_bytes(int d, const int* cap, int dtype);
size_t wgrad_ws_bytes(int d, const int32_t* w_cap);
int run_conv_backward_w(const TensorDev& w, int dtype, const void* f, const void* gy, void* gf,
                        const TensorDev& gw, void* ws, hipStream_t s);
int run_full_adjoint(const TensorDev& f, int dtype, const void* g, const TensorDev& gr, void* ws,
                     hipStream_t s);
constexpr int kDotPartials = 512;
int run_dot(int dtype, const void* a, const void* b, long long n, double* part, double* out,
            hipStream_t s);
size_t sinc_sums_ws_bytes();
int run_sinc_sums(double B, int nk, void* ws, double** consts, hipStream_t s);

}  // namespace qtt

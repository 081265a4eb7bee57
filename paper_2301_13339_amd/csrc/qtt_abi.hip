// extern "C" entry points of libqtt: argument checks, workspace planning and
// dispatch to the HIP kernels.  See include/qtt.h for the contract.
#include <math.h>
#include <string.h>

#include "qtt_internal.hpp"

namespace qtt {

static thread_local char g_hip_err[256] = "";

void set_hip_error(hipError_t e) {
  const char* s = hipGetErrorString(e);
  strncpy(g_hip_err, s ? s : "unknown HIP error", sizeof(g_hip_err) - 1);
  g_hip_err[sizeof(g_hip_err) - 1] = 0;
}

// ------------------------------------------------------------ launch probe
struct ProbeState {
  int cls = 0;
  int cap = 0;
  int n = 0;
  hipEvent_t* ev = nullptr;
};
static ProbeState g_probe;

void probe_pre(int cls, hipStream_t s) {
  if (g_probe.cls != cls || g_probe.n >= g_probe.cap) return;
  hipEventRecord(g_probe.ev[2 * g_probe.n], s);
}

void probe_post(int cls, hipStream_t s) {
  if (g_probe.cls != cls || g_probe.n >= g_probe.cap) return;
  hipEventRecord(g_probe.ev[2 * g_probe.n + 1], s);
  ++g_probe.n;
}

static void probe_free() {
  if (g_probe.ev) {
    for (int i = 0; i < 2 * g_probe.cap; ++i) hipEventDestroy(g_probe.ev[i]);
    delete[] g_probe.ev;
  }
  g_probe = ProbeState();
}

static int eff_rank(int max_rank) {
  return (max_rank <= 0 || max_rank > kMaxRank) ? kMaxRank : max_rank;
}

static bool dtype_ok(int dt) { return dt == QTT_F32 || dt == QTT_F64; }

constexpr int kMaxModes = 30;  // largest d for operations on full arrays (2^30 samples)

static void caps_decompose(int d, int rcap, int32_t* cap) {
  for (int k = 0; k <= d; ++k) {
    long long c = rcap;
    const long long lo = 1LL << (k < 40 ? k : 40), hi = 1LL << ((d - k) < 40 ? (d - k) : 40);
    if (lo < c) c = lo;
    if (hi < c) c = hi;
    cap[k] = (k == 0 || k == d) ? 1 : (int32_t)c;
  }
}

static size_t core_elems_of(int d, const int32_t* cap) {
  size_t s = 0;
  for (int k = 0; k < d; ++k) s += (size_t)cap[k] * 2 * (size_t)cap[k + 1];
  return s;
}

// the tensor descriptor is usable as an output with at least the given capacities
static int check_tensor(const qtt_tensor* t, int d, int dtype, const int32_t* need) {
  if (!t || t->d != d || t->dtype != dtype || !t->ranks || !t->cores) return QTT_EINVAL;
  if (t->cap[0] != 1 || t->cap[d] != 1) return QTT_EINVAL;
  for (int k = 0; k <= d; ++k)
    if (t->cap[k] < need[k]) return QTT_ENOSPC;
  return QTT_OK;
}

static int check_tensor_in(const qtt_tensor* t) {
  if (!t || t->d < 1 || t->d > kMaxModes + 1 || !dtype_ok(t->dtype) || !t->ranks || !t->cores)
    return QTT_EINVAL;
  if (t->cap[0] != 1 || t->cap[t->d] != 1) return QTT_EINVAL;
  for (int k = 1; k < t->d; ++k)
    if (t->cap[k] < 1) return QTT_EINVAL;
  return QTT_OK;
}

}  // namespace qtt

using namespace qtt;

extern "C" {

size_t qtt_core_elems(int d, const int32_t* cap) {
  if (d < 1 || d > QTT_MAXD || !cap) return 0;
  return core_elems_of(d, cap);
}

const char* qtt_strerror(int code) {
  switch (code) {
    case QTT_OK: return "ok";
    case QTT_EINVAL: return "invalid argument";
    case QTT_ENOSPC: return "workspace or tensor capacity too small";
    case QTT_ENOTSUP: return "unsupported size or option";
    case QTT_EHIP: return "HIP runtime error";
    case QTT_STATUS_NONFINITE: return "input held a non-finite value";
    case QTT_STATUS_RANKCAP: return "an eps-rank exceeded the rank capacity";
    case QTT_STATUS_FFT_RANK: return "a QTT-FFT input rank exceeded QTT_FFT_MAX_RANK";
    case QTT_STATUS_NONFINITE | QTT_STATUS_RANKCAP:
      return "non-finite input; an eps-rank exceeded the rank capacity";
    default: return "unknown code";
  }
}

const char* qtt_last_hip_error(void) { return g_hip_err; }

int qtt_probe_start(int cls, int max_launches) {
  if (cls < QTT_K_LEVEL_GRAM || cls > QTT_K_QFFT_HADAMARD || max_launches < 1 || max_launches > (1 << 20))
    return QTT_EINVAL;
  probe_free();
  g_probe.ev = new hipEvent_t[2 * (size_t)max_launches];
  for (int i = 0; i < 2 * max_launches; ++i) {
    const hipError_t e = hipEventCreate(&g_probe.ev[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) hipEventDestroy(g_probe.ev[j]);
      delete[] g_probe.ev;
      g_probe = ProbeState();
      set_hip_error(e);
      return QTT_EHIP;
    }
  }
  g_probe.cap = max_launches;
  g_probe.cls = cls;
  return QTT_OK;
}

int qtt_probe_stop(double* total_ms, int* launches) {
  double tot = 0.0;
  const int n = g_probe.n;
  for (int i = 0; i < n; ++i) {
    const hipError_t e = hipEventSynchronize(g_probe.ev[2 * i + 1]);
    if (e != hipSuccess) {
      set_hip_error(e);
      probe_free();
      return QTT_EHIP;
    }
    float ms = 0.f;
    hipEventElapsedTime(&ms, g_probe.ev[2 * i], g_probe.ev[2 * i + 1]);
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = n;
  probe_free();
  return QTT_OK;
}

// ------------------------------------------------------------- decompose
int qtt_query_decompose(int d, int max_rank, int dtype, int32_t* cap, size_t* ws_bytes,
                        size_t* core_elems) {
  if (d < 1 || d > kMaxModes + 1 || max_rank < 0 || !dtype_ok(dtype)) return QTT_EINVAL;
  DecompPlan p;
  plan_decompose(d, eff_rank(max_rank), dtype, nullptr, &p);
  int32_t c[QTT_MAXD + 1];
  caps_decompose(d, eff_rank(max_rank), c);
  if (cap) memcpy(cap, c, sizeof(int32_t) * (d + 1));
  if (ws_bytes) *ws_bytes = p.ws_bytes;
  if (core_elems) *core_elems = core_elems_of(d, c);
  return QTT_OK;
}

static int decompose_common(const Source& src, int D, int dtype, double eps, int max_rank,
                            qtt_tensor* out, double* sv, void* ws, size_t ws_bytes,
                            void* stream, double delta = 0.0) {
  if (D < 1 || D > kMaxModes + 1 || !dtype_ok(dtype) || !(eps >= 0.0) || !isfinite(eps) ||
      max_rank < 0 || !(delta >= 0.0 && delta < 1.0))
    return QTT_EINVAL;
  if (!ws) return QTT_EINVAL;
  DecompPlan p;
  plan_decompose(D, eff_rank(max_rank), dtype, nullptr, &p);
  if (ws_bytes < p.ws_bytes) return QTT_ENOSPC;
  int32_t need[QTT_MAXD + 1];
  caps_decompose(D, eff_rank(max_rank), need);
  const int rc = check_tensor(out, D, dtype, need);
  if (rc) return rc;
  plan_decompose(D, eff_rank(max_rank), dtype, ws, &p);
  TensorDev td = make_dev(out);
  return run_decompose(p, src, eps, td, sv, static_cast<hipStream_t>(stream), delta);
}

int qtt_decompose(const void* x, int d, int dtype, double eps, int max_rank, qtt_tensor* out,
                  double* sv, void* ws, size_t ws_bytes, void* stream) {
  if (!x) return QTT_EINVAL;
  Source src{x, 0, 0.0, 0};
  return decompose_common(src, d, dtype, eps, max_rank, out, sv, ws, ws_bytes, stream);
}

int qtt_decompose_dropoff(const void* x, int d, int dtype, double eps, double delta, int max_rank,
                          qtt_tensor* out, double* sv, void* ws, size_t ws_bytes, void* stream) {
  if (!x) return QTT_EINVAL;
  Source src{x, 0, 0.0, 0};
  return decompose_common(src, d, dtype, eps, max_rank, out, sv, ws, ws_bytes, stream, delta);
}

// ------------------------------------------------------ general mode sizes
static int modes_args_ok(int K, int M, int max_rank, int method, int oversample) {
  if (K < 1 || M < 2 || M > kModesMaxM || max_rank < 0 || (method != 0 && method != 1))
    return 0;
  double n = 1.0;
  for (int k = 0; k < K; ++k) n *= M;
  if (n > 2147483648.0) return 0;  // at most 2^31 entries
  if (method == 1) {
    int32_t cap[QTT_MAXD + 1];
    if (K > QTT_MAXD) return 0;
    const int R = modes_caps(K, M, max_rank, cap);
    if (max_rank <= 0 || oversample < 0 || R + oversample > 64) return 0;
  }
  return K <= QTT_MAXD;
}

int qtt_query_decompose_modes(int K, int M, int max_rank, int method, int oversample,
                              int32_t* cap, size_t* ws_bytes, size_t* core_elems) {
  if (!modes_args_ok(K, M, max_rank, method, oversample)) return QTT_EINVAL;
  int32_t c[QTT_MAXD + 1];
  modes_caps(K, M, max_rank, c);
  if (cap) memcpy(cap, c, sizeof(int32_t) * (K + 1));
  if (ws_bytes) *ws_bytes = modes_ws_bytes(K, M, method, oversample);
  if (core_elems) {
    size_t e = 0;
    for (int k = 0; k < K; ++k) e += (size_t)c[k] * M * c[k + 1];
    *core_elems = e;
  }
  return QTT_OK;
}

int qtt_decompose_modes(const double* x, int K, int M, double eps, int max_rank, int method,
                        int oversample, uint64_t seed, const int32_t* cap, int32_t* ranks,
                        double* cores, int32_t* status, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!x || !cap || !ranks || !cores || !ws || !(eps >= 0.0) || !isfinite(eps) ||
      !modes_args_ok(K, M, max_rank, method, oversample))
    return QTT_EINVAL;
  if (ws_bytes < modes_ws_bytes(K, M, method, oversample)) return QTT_ENOSPC;
  int32_t need[QTT_MAXD + 1];
  modes_caps(K, M, max_rank, need);
  for (int k = 0; k <= K; ++k)
    if (cap[k] < need[k]) return QTT_ENOSPC;
  for (int k = 0; k <= K; ++k)
    if (cap[k] != need[k]) return QTT_EINVAL;  // the core offsets follow the query's capacities
  // the library's capacity (QTT_MAX_RANK, lowered to 128 / M) decides when it
  // is below the caller's cap; only then is a binding cap reported
  const int lib_cap = (128 / M) < QTT_MAX_RANK ? 128 / M : QTT_MAX_RANK;
  const int lib_capped = (max_rank == 0 || max_rank > lib_cap) ? 1 : 0;
  return run_decompose_modes(x, K, M, eps, method, oversample, seed, cap, ranks, cores, status,
                             lib_capped, ws, static_cast<hipStream_t>(stream));
}

int qtt_kernel_sinc(int d, double B, double eps_w, int dtype, qtt_tensor* w_out, void* ws,
                    size_t ws_bytes, void* stream) {
  if (d < 1 || d > kMaxModes || !(B > 0.0) || !isfinite(B)) return QTT_EINVAL;
  Source src{nullptr, 1, B, d};
  return decompose_common(src, d + 1, dtype, eps_w, 0, w_out, nullptr, ws, ws_bytes, stream);
}

// ------------------------------------------------------------------ conv
static int conv_caps(int d, int n_axes, const int32_t* axis_modes, const int32_t* f_cap,
                     const int32_t* const* w_caps, int32_t* y_cap) {
  if (n_axes < 1 || n_axes > 2 || !axis_modes || !f_cap || !w_caps) return QTT_EINVAL;
  int sum = 0;
  for (int a = 0; a < n_axes; ++a) {
    if (axis_modes[a] < 1 || !w_caps[a]) return QTT_EINVAL;
    sum += axis_modes[a];
  }
  if (sum != d) return QTT_EINVAL;
  int k = 0;
  y_cap[0] = 1;
  for (int a = 0; a < n_axes; ++a) {
    for (int kap = 1; kap <= axis_modes[a]; ++kap, ++k) {
      const long long fc = f_cap[k + 1];
      const long long c = (kap == axis_modes[a]) ? fc : 2LL * w_caps[a][kap] * fc;
      if (c > (1LL << 30)) return QTT_ENOTSUP;
      y_cap[k + 1] = (int32_t)c;
    }
  }
  y_cap[d] = 1;
  return QTT_OK;
}

int qtt_query_conv(int d, int n_axes, const int32_t* axis_modes, const int32_t* f_cap,
                   const int32_t* const* w_caps, int dtype, int32_t* y_cap, size_t* ws_bytes,
                   size_t* core_elems) {
  if (d < 1 || d > kMaxModes || !dtype_ok(dtype)) return QTT_EINVAL;
  int32_t yc[QTT_MAXD + 1];
  const int rc = conv_caps(d, n_axes, axis_modes, f_cap, w_caps, yc);
  if (rc) return rc;
  if (y_cap) memcpy(y_cap, yc, sizeof(int32_t) * (d + 1));
  if (ws_bytes) *ws_bytes = 0;
  if (core_elems) *core_elems = core_elems_of(d, yc);
  return QTT_OK;
}

int qtt_conv(const qtt_tensor* f, const qtt_tensor* w, int n_axes, const int32_t* axis_modes,
             qtt_tensor* y, void* ws, size_t ws_bytes, void* stream) {
  (void)ws;
  (void)ws_bytes;
  if (check_tensor_in(f) || !w || n_axes < 1 || n_axes > 2 || !axis_modes) return QTT_EINVAL;
  const int d = f->d;
  if (d > kMaxModes) return QTT_EINVAL;
  const int32_t* wc[2] = {nullptr, nullptr};
  for (int a = 0; a < n_axes; ++a) {
    if (check_tensor_in(&w[a]) || w[a].dtype != f->dtype || w[a].d != axis_modes[a] + 1)
      return QTT_EINVAL;
    wc[a] = w[a].cap;
  }
  int32_t yc[QTT_MAXD + 1];
  int rc = conv_caps(d, n_axes, axis_modes, f->cap, wc, yc);
  if (rc) return rc;
  rc = check_tensor(y, d, f->dtype, yc);
  if (rc) return rc;
  TensorDev fd = make_dev(f), yd = make_dev(y);
  TensorDev wd[2];
  for (int a = 0; a < n_axes; ++a) wd[a] = make_dev(&w[a]);
  return run_conv(fd, wd, n_axes, axis_modes, yd, f->dtype, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------------------ full
int qtt_query_full(int d, const int32_t* cap, int dtype, size_t* ws_bytes) {
  if (d < 1 || d > kMaxModes || !cap || !dtype_ok(dtype)) return QTT_EINVAL;
  void* bufs[4];
  size_t b = 0;
  plan_full(d, cap, dtype, nullptr, &b, bufs);
  if (ws_bytes) *ws_bytes = b;
  return QTT_OK;
}

int qtt_full(const qtt_tensor* t, void* out, void* ws, size_t ws_bytes, void* stream) {
  if (check_tensor_in(t) || !out || t->d > kMaxModes) return QTT_EINVAL;
  size_t need = 0;
  void* bufs[4];
  plan_full(t->d, t->cap, t->dtype, nullptr, &need, bufs);
  if (need > 0 && (!ws || ws_bytes < need)) return need > ws_bytes ? QTT_ENOSPC : QTT_EINVAL;
  TensorDev td = make_dev(t);
  return run_full(td, t->dtype, out, ws, static_cast<hipStream_t>(stream));
}

// ----------------------------------------------------------------- round
struct RoundPlan {
  void* yfull;
  void* full_ws;
  size_t full_bytes;
  void* dec_ws;
  size_t dec_bytes;
  size_t total;
};

static void plan_round(int d, const int32_t* y_cap, int rcap, int dtype, int ell, void* ws,
                       RoundPlan* rp) {
  Arena ar(ws);
  const size_t es = elem_size(dtype);
  rp->yfull = ar.take<char>(((size_t)1 << d) * es);
  void* bufs[4];
  size_t fb = 0;
  plan_full(d, y_cap, dtype, nullptr, &fb, bufs);
  rp->full_ws = ar.take<char>(fb);
  rp->full_bytes = fb;
  size_t db;
  if (ell > 0) {
    db = sketch_ws_bytes(d, dtype, ell);
  } else {
    DecompPlan p;
    plan_decompose(d, rcap, dtype, nullptr, &p);
    db = p.ws_bytes;
  }
  rp->dec_ws = ar.take<char>(db);
  rp->dec_bytes = db;
  rp->total = ar.size();
}

// ell = 0: exact rounding; otherwise the sketch width
static int query_round_common(int d, const int32_t* y_cap, int max_rank, int dtype, int ell,
                              int32_t* z_cap, size_t* ws_bytes, size_t* core_elems) {
  if (d < 1 || d > kMaxModes || !y_cap || !dtype_ok(dtype) || max_rank < 0) return QTT_EINVAL;
  RoundPlan rp;
  plan_round(d, y_cap, eff_rank(max_rank), dtype, ell, nullptr, &rp);
  int32_t zc[QTT_MAXD + 1];
  caps_decompose(d, eff_rank(max_rank), zc);
  if (z_cap) memcpy(z_cap, zc, sizeof(int32_t) * (d + 1));
  if (ws_bytes) *ws_bytes = rp.total;
  if (core_elems) *core_elems = core_elems_of(d, zc);
  return QTT_OK;
}

int qtt_query_round(int d, const int32_t* y_cap, int max_rank, int dtype, int method,
                    int32_t* z_cap, size_t* ws_bytes, size_t* core_elems) {
  if (method < QTT_ROUND_EXACT || method > QTT_ROUND_SKETCH_BF16) return QTT_EINVAL;
  return query_round_common(d, y_cap, max_rank, dtype,
                            method == QTT_ROUND_EXACT ? 0 : QTT_SKETCH_ELL, z_cap, ws_bytes,
                            core_elems);
}

int qtt_query_round_sketch(int d, const int32_t* y_cap, int max_rank, int dtype, int ell,
                           int32_t* z_cap, size_t* ws_bytes, size_t* core_elems) {
  if (ell < 2 || ell > QTT_SKETCH_MAX_ELL) return QTT_EINVAL;
  return query_round_common(d, y_cap, max_rank, dtype, ell, z_cap, ws_bytes, core_elems);
}

static int round_common(const qtt_tensor* y, double eps, int max_rank, int ell, int bf16,
                        uint64_t seed, qtt_tensor* z, void* ws, size_t ws_bytes, void* stream) {
  if (check_tensor_in(y) || y->d > kMaxModes || !(eps >= 0.0) || !isfinite(eps) || max_rank < 0 ||
      !ws)
    return QTT_EINVAL;
  const int d = y->d;
  if (d < 2) ell = 0;  // one mode: nothing to truncate, the exact path copies
  RoundPlan rp;
  plan_round(d, y->cap, eff_rank(max_rank), y->dtype, ell, nullptr, &rp);
  if (ws_bytes < rp.total) return QTT_ENOSPC;
  int32_t zc[QTT_MAXD + 1];
  caps_decompose(d, eff_rank(max_rank), zc);
  int rc = check_tensor(z, d, y->dtype, zc);
  if (rc) return rc;
  plan_round(d, y->cap, eff_rank(max_rank), y->dtype, ell, ws, &rp);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TensorDev yd = make_dev(y);
  rc = run_full(yd, y->dtype, rp.yfull, rp.full_ws, st);
  if (rc) return rc;
  TensorDev zd = make_dev(z);
  if (ell > 0) {
    int capi[QTT_MAXD + 1];
    for (int k = 0; k <= d; ++k) capi[k] = zc[k];
    return run_round_sketch(y->dtype, bf16, rp.yfull, d, eps, capi, ell, seed, zd, rp.dec_ws, st);
  }
  DecompPlan p;
  plan_decompose(d, eff_rank(max_rank), y->dtype, rp.dec_ws, &p);
  Source src{rp.yfull, 0, 0.0, 0};
  return run_decompose(p, src, eps, zd, nullptr, st);
}

int qtt_round(const qtt_tensor* y, double eps, int max_rank, int method, uint64_t seed,
              qtt_tensor* z, void* ws, size_t ws_bytes, void* stream) {
  if (method < QTT_ROUND_EXACT || method > QTT_ROUND_SKETCH_BF16) return QTT_EINVAL;
  const int ell = method == QTT_ROUND_EXACT ? 0 : QTT_SKETCH_ELL;
  return round_common(y, eps, max_rank, ell, method == QTT_ROUND_SKETCH_BF16, seed, z, ws,
                      ws_bytes, stream);
}

int qtt_round_sketch(const qtt_tensor* y, double eps, int max_rank, int ell, int bf16,
                     uint64_t seed, qtt_tensor* z, void* ws, size_t ws_bytes, void* stream) {
  if (ell < 2 || ell > QTT_SKETCH_MAX_ELL || (bf16 != 0 && bf16 != 1)) return QTT_EINVAL;
  return round_common(y, eps, max_rank, ell, bf16, seed, z, ws, ws_bytes, stream);
}

// --------------------------------------------------------------- adjoint
static int wcap_ok(const int32_t* w_cap, int D) {
  if (!w_cap || w_cap[0] != 1 || w_cap[D] != 1) return 0;
  for (int k = 1; k < D; ++k)
    if (w_cap[k] < 1 || w_cap[k] > QTT_MAX_RANK) return 0;
  return 1;
}

int qtt_query_toeplitz(int d, const int32_t* w_cap, int dtype, size_t* ws_bytes) {
  if (d < 1 || d > kMaxModes || !dtype_ok(dtype) || !wcap_ok(w_cap, d + 1)) return QTT_EINVAL;
  if (ws_bytes) *ws_bytes = toeplitz_ws_elems(d, w_cap) * sizeof(double);
  return QTT_OK;
}

int qtt_toeplitz_apply(const qtt_tensor* w, const void* x, void* y, int transpose, void* ws,
                       size_t ws_bytes, void* stream) {
  if (check_tensor_in(w) || w->d < 2 || !x || !y || (transpose != 0 && transpose != 1))
    return QTT_EINVAL;
  const int d = w->d - 1;
  if (d > kMaxModes || !wcap_ok(w->cap, w->d)) return QTT_EINVAL;
  const size_t need = toeplitz_ws_elems(d, w->cap) * sizeof(double);
  if (!ws || ws_bytes < need) return ws ? QTT_ENOSPC : QTT_EINVAL;
  TensorDev wd = make_dev(w);
  return run_toeplitz(wd, w->dtype, x, y, transpose, ws, static_cast<hipStream_t>(stream));
}

int qtt_query_kernel_sinc_dB(int d, int dtype, int32_t* cap, size_t* ws_bytes,
                             size_t* core_elems) {
  if (d < 1 || d > kMaxModes) return QTT_EINVAL;
  size_t b = 0;
  const int rc = qtt_query_decompose(d + 1, 0, dtype, cap, &b, core_elems);
  if (rc) return rc;
  if (ws_bytes) *ws_bytes = b + sinc_sums_ws_bytes();
  return QTT_OK;
}

int qtt_kernel_sinc_dB(int d, double B, double eps_w, int dtype, qtt_tensor* w_out, void* ws,
                       size_t ws_bytes, void* stream) {
  if (d < 1 || d > kMaxModes || !(B > 0.0) || !isfinite(B) || !ws) return QTT_EINVAL;
  const size_t sb = sinc_sums_ws_bytes();
  if (ws_bytes < sb) return QTT_ENOSPC;
  // validate everything before the first launch
  {
    DecompPlan p;
    if (d + 1 > kMaxModes + 1 || !dtype_ok(dtype) || !(eps_w >= 0.0) || !isfinite(eps_w))
      return QTT_EINVAL;
    plan_decompose(d + 1, eff_rank(0), dtype, nullptr, &p);
    if (ws_bytes - sb < p.ws_bytes) return QTT_ENOSPC;
    int32_t need[QTT_MAXD + 1];
    caps_decompose(d + 1, eff_rank(0), need);
    const int rc = check_tensor(w_out, d + 1, dtype, need);
    if (rc) return rc;
  }
  double* consts = nullptr;
  int rc = run_sinc_sums(B, d, ws, &consts, static_cast<hipStream_t>(stream));
  if (rc) return rc;
  Source src{consts, 2, B, d};
  return decompose_common(src, d + 1, dtype, eps_w, 0, w_out, nullptr,
                          static_cast<char*>(ws) + sb, ws_bytes - sb, stream);
}

int qtt_query_full_adjoint(int d, const int32_t* cap, int dtype, size_t* ws_bytes) {
  if (d < 1 || d > kMaxModes || !cap || !dtype_ok(dtype)) return QTT_EINVAL;
  for (int k = 0; k <= d; ++k)
    if (cap[k] < 1 || cap[k] > QTT_MAX_RANK) return QTT_EINVAL;
  if (ws_bytes) *ws_bytes = full_adjoint_ws_bytes(d, cap, dtype);
  return QTT_OK;
}

static int grad_tensor_ok(const qtt_tensor* f, const qtt_tensor* g) {
  if (!g || g->d != f->d || g->dtype != f->dtype || !g->ranks || !g->cores) return QTT_EINVAL;
  for (int k = 0; k <= f->d; ++k)
    if (g->cap[k] != f->cap[k]) return QTT_EINVAL;
  return QTT_OK;
}

int qtt_full_adjoint(const qtt_tensor* f, const void* g, qtt_tensor* grad, void* ws,
                     size_t ws_bytes, void* stream) {
  if (check_tensor_in(f) || f->d > kMaxModes || !g || grad_tensor_ok(f, grad)) return QTT_EINVAL;
  for (int k = 0; k <= f->d; ++k)
    if (f->cap[k] > QTT_MAX_RANK) return QTT_ENOTSUP;
  const size_t need = full_adjoint_ws_bytes(f->d, f->cap, f->dtype);
  if (!ws || ws_bytes < need) return ws ? QTT_ENOSPC : QTT_EINVAL;
  TensorDev fd = make_dev(f), gd = make_dev(grad);
  return run_full_adjoint(fd, f->dtype, g, gd, ws, static_cast<hipStream_t>(stream));
}

struct BwdPlan {
  void* ffull;
  void* gf;
  void* z;
  void* toep_ws;
  void* full_ws;
  void* adj_ws;
  void* wg_ws;
  double* dot_part;
  size_t total;
};

static void plan_backward(int d, const int32_t* f_cap, const int32_t* w_cap,
                          const int32_t* wdb_cap, int want_w, int dtype, void* ws, BwdPlan* p) {
  Arena ar(ws);
  const size_t es = elem_size(dtype);
  const size_t N = (size_t)1 << d;
  p->ffull = ar.take<char>(N * es);
  p->gf = ar.take<char>(N * es);
  p->z = wdb_cap ? ar.take<char>(N * es) : nullptr;
  size_t te = toeplitz_ws_elems(d, w_cap);
  if (wdb_cap) {
    const size_t t2 = toeplitz_ws_elems(d, wdb_cap);
    if (t2 > te) te = t2;
  }
  p->toep_ws = ar.take<double>(te);
  void* bufs[4];
  size_t fb = 0;
  plan_full(d, f_cap, dtype, nullptr, &fb, bufs);
  p->full_ws = ar.take<char>(fb > 0 ? fb : 1);
  p->adj_ws = ar.take<char>(full_adjoint_ws_bytes(d, f_cap, dtype));
  p->wg_ws = want_w ? ar.take<char>(wgrad_ws_bytes(d, w_cap)) : nullptr;
  p->dot_part = ar.take<double>(kDotPartials + 8);
  p->total = ar.size();
}

int qtt_query_conv_full_backward(int d, const int32_t* f_cap, const int32_t* w_cap,
                                 const int32_t* wdb_cap, int want_w, int dtype,
                                 size_t* ws_bytes) {
  if (d < 1 || d > kMaxModes || !f_cap || !dtype_ok(dtype) || !wcap_ok(w_cap, d + 1) ||
      (wdb_cap && !wcap_ok(wdb_cap, d + 1)) || (want_w != 0 && want_w != 1))
    return QTT_EINVAL;
  for (int k = 0; k <= d; ++k)
    if (f_cap[k] < 1 || f_cap[k] > QTT_MAX_RANK) return QTT_EINVAL;
  BwdPlan p;
  plan_backward(d, f_cap, w_cap, wdb_cap, want_w, dtype, nullptr, &p);
  if (ws_bytes) *ws_bytes = p.total;
  return QTT_OK;
}

int qtt_conv_full_backward(const qtt_tensor* f, const qtt_tensor* w, const qtt_tensor* w_dB,
                           const void* grad_y, qtt_tensor* grad_f, qtt_tensor* grad_w,
                           double* grad_B, void* ws, size_t ws_bytes, void* stream) {
  if (check_tensor_in(f) || f->d > kMaxModes || check_tensor_in(w) || !grad_y ||
      grad_tensor_ok(f, grad_f))
    return QTT_EINVAL;
  const int d = f->d;
  if (w->d != d + 1 || w->dtype != f->dtype || !wcap_ok(w->cap, d + 1)) return QTT_EINVAL;
  if (w_dB && (check_tensor_in(w_dB) || w_dB->d != d + 1 || w_dB->dtype != f->dtype ||
               !wcap_ok(w_dB->cap, d + 1)))
    return QTT_EINVAL;
  if ((w_dB == nullptr) != (grad_B == nullptr)) return QTT_EINVAL;
  if (grad_w && grad_tensor_ok(w, grad_w)) return QTT_EINVAL;
  for (int k = 0; k <= d; ++k)
    if (f->cap[k] > QTT_MAX_RANK) return QTT_ENOTSUP;
  const int want_w = grad_w ? 1 : 0;
  BwdPlan p;
  plan_backward(d, f->cap, w->cap, w_dB ? w_dB->cap : nullptr, want_w, f->dtype, nullptr, &p);
  if (!ws || ws_bytes < p.total) return ws ? QTT_ENOSPC : QTT_EINVAL;
  plan_backward(d, f->cap, w->cap, w_dB ? w_dB->cap : nullptr, want_w, f->dtype, ws, &p);
  hipStream_t st = static_cast<hipStream_t>(stream);
  TensorDev fd = make_dev(f), wd = make_dev(w), gd = make_dev(grad_f);
  // the core chain is recomputed here rather than kept from the forward
  int rc = run_full(fd, f->dtype, p.ffull, p.full_ws, st);
  if (rc) return rc;
  if (grad_w) {
    // T(w)^T grad_y and the kernel-core gradients in one pair of sweeps
    TensorDev gwd = make_dev(grad_w);
    rc = run_conv_backward_w(wd, f->dtype, p.ffull, grad_y, p.gf, gwd, p.wg_ws, st);
  } else {
    rc = run_toeplitz(wd, f->dtype, grad_y, p.gf, 1, p.toep_ws, st);
  }
  if (rc) return rc;
  rc = run_full_adjoint(fd, f->dtype, p.gf, gd, p.adj_ws, st);
  if (rc) return rc;
  if (w_dB) {
    TensorDev bd = make_dev(w_dB);
    rc = run_toeplitz(bd, f->dtype, p.ffull, p.z, 0, p.toep_ws, st);
    if (rc) return rc;
    rc = run_dot(f->dtype, grad_y, p.z, 1LL << d, p.dot_part, grad_B, st);
  }
  return rc;
}

}  // extern "C"

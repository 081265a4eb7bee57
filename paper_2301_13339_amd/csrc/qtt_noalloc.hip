// Allocation-free reconstruction: qtt_full with the half-chain interface
// matrices in a fixed device array of the library instead of a caller
// workspace.  For callers that cannot allocate device memory (code under
// stream capture, serving loops, harnesses that forbid hipMalloc).
//
// The array lives in this translation unit as a file-scope __device__
// variable.  Host code never passes its name to a kernel: the name is a
// host-side shadow, not a device address.  The first call on a device looks
// up the device address with hipGetSymbolAddress (that device current) and
// keeps it; every later call on that device uses the stored pointer.
#include <mutex>

#include "qtt_internal.hpp"

namespace qtt {

// Largest interface-matrix storage one call may use (bytes).
constexpr size_t kNoAllocScratchBytes = size_t(QTT_NOALLOC_SCRATCH_MIB) << 20;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
static int scratch_ptr(void** out) {
  int dev = 0;
  QTT_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return QTT_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    QTT_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return QTT_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QTT_OK;
}

}  // namespace qtt

using namespace qtt;

extern "C" int qtt_full_noalloc(const qtt_tensor* t, void* out, void* stream) {
  if (!t || !out || t->d < 1 || t->d > 30 || (t->dtype != QTT_F32 && t->dtype != QTT_F64) ||
      !t->ranks || !t->cores)
    return QTT_EINVAL;
  if (t->cap[0] != 1 || t->cap[t->d] != 1) return QTT_EINVAL;
  for (int k = 1; k < t->d; ++k)
    if (t->cap[k] < 1) return QTT_EINVAL;
  size_t need = 0;
  void* bufs[4];
  plan_full(t->d, t->cap, t->dtype, nullptr, &need, bufs);
  if (need > kNoAllocScratchBytes) return QTT_ENOSPC;
  void* ws = nullptr;
  int rc = scratch_ptr(&ws);
  if (rc) return rc;
  TensorDev td = make_dev(t);
  return run_full(td, t->dtype, out, ws, static_cast<hipStream_t>(stream));
}

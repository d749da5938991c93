// qcoll_eval without a caller workspace and without any allocation: the
// pipeline's scratch (spectra, per-node half spectra, per-term volumes) lives
// in one file-scope device array of fixed size, and the batch runs in chunks
// small enough for it.
//
// In host code the array's name is only a stand-in for the symbol; its device
// address is taken once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "qcoll_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;   // 256 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

qcoll_status nfail(qcoll_status s, const std::string &m) {
  qcoll::set_error(m);
  return s;
}

// device address of this device's copy of the array (dev is current)
qcoll_status scratch_ptr(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return nfail(QCOLL_ENOTSUP, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return nfail(QCOLL_EDEVICE, std::string("hipGetSymbolAddress failed for the scratch array: ") +
                                      hipGetErrorString(e));
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return QCOLL_OK;
}

}  // namespace

extern "C" qcoll_status qcoll_eval_noalloc(qcoll_plan plan, int64_t batch, const double *f, double *Q,
                                           void *stream) {
  if (!plan) return nfail(QCOLL_EINVAL, "plan is NULL");
  if (batch < 0) return nfail(QCOLL_EINVAL, "batch must be >= 0");
  if (batch == 0) return QCOLL_OK;
  if (!f || !Q) return nfail(QCOLL_EINVAL, "f and Q must be non-NULL");
  const qcoll::Plan &p = plan->p;
  const long n3 = p.n3();
  if ((const void *)f < (const void *)(Q + batch * n3) && (const void *)Q < (const void *)(f + batch * n3))
    return nfail(QCOLL_EINVAL, "Q must not overlap f");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return nfail(QCOLL_EDEVICE, "hipGetDevice failed");
  if (dev != p.device) return nfail(QCOLL_EINVAL, "current device differs from the plan's device");
  // items per chunk: the plan's chunk (default 64), reduced until one chunk's
  // workspace fits the array (the workspace grows with the chunk)
  const long want = std::min<long>(batch, p.chunk > 0 ? p.chunk : 64);
  if (qcoll::make_layout(p, batch, 0, 1).total > kScratchBytes)
    return nfail(QCOLL_EWORKSPACE, "one item of this plan needs " +
                                       std::to_string(qcoll::make_layout(p, batch, 0, 1).total) +
                                       " bytes of scratch; qcoll_eval_noalloc holds " +
                                       std::to_string(kScratchBytes) + " (use qcoll_eval with a workspace)");
  long lo = 1, hi = want;   // largest chunk in [1, want] that fits
  while (lo < hi) {
    const long mid = (lo + hi + 1) / 2;
    if (qcoll::make_layout(p, batch, 0, mid).total <= kScratchBytes) lo = mid;
    else hi = mid - 1;
  }
  void *ws = nullptr;
  qcoll_status st = scratch_ptr(dev, &ws);
  if (st != QCOLL_OK) return st;
  const qcoll::Layout lay = qcoll::make_layout(p, batch, 0, lo);
  return qcoll::launch_eval(p, batch, f, Q, ws, lay, static_cast<hipStream_t>(stream));
}

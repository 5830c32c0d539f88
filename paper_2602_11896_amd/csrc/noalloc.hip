// JTFS forward without any allocation: the workspace is a file-scope device array.
//
// jtfs_forward needs a caller workspace of ws_shared_forward bytes per call (the
// stage-boundary tensors, pooled partials and two-pass FFT scratch of one signal).
// jtfs_forward_noalloc takes it from `scratch` below instead, so a caller that may not
// allocate (code under HIP graph capture, a tight serving loop) passes only x and S.
// The array's device address is resolved once per device by jtfs_plan_prepare; every
// call on a device shares that device's array and leaves its contents behind, so calls
// that overlap on one device race. No kernel of the forward reads workspace memory it has
// not written in the same call, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/jtfs.h"
#include "abi_internal.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[JTFS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device; null: unresolved

}  // namespace

extern "C" {

jtfs_status jtfs_plan_prepare(jtfs_plan_t plan) {
  if (!plan) return jtfs::report(JTFS_ERR_ARG, "NULL plan");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return jtfs::report(JTFS_ERR_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxDevices) return jtfs::report(JTFS_ERR_UNSUPPORTED, "device index beyond 63");
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return jtfs::report(JTFS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_scratch[dev] = ptr;
    }
  }
  return jtfs::prepare_tables(plan);
}

jtfs_status jtfs_forward_noalloc(jtfs_plan_t plan, const float* x, float* S, jtfs_stream_t stream) {
  if (!plan || !x || !S) return jtfs::report(JTFS_ERR_ARG, "NULL argument");
  const size_t need = jtfs::shared_forward_bytes(plan);
  if (need > JTFS_NOALLOC_SCRATCH_BYTES)
    return jtfs::report(JTFS_ERR_WORKSPACE, "the plan's forward needs " + std::to_string(need) +
                                                " workspace bytes, beyond the " +
                                                std::to_string(static_cast<size_t>(JTFS_NOALLOC_SCRATCH_BYTES)) +
                                                " of the no-allocation scratch");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return jtfs::report(JTFS_ERR_HIP, "hipGetDevice failed");
  void* ws = nullptr;
  if (dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> lock(g_mu);
    ws = g_scratch[dev];
  }
  if (!ws) return jtfs::report(JTFS_ERR_ARG, "no scratch on this device: call jtfs_plan_prepare first");
  return jtfs::forward_prepared(plan, x, S, ws, static_cast<hipStream_t>(stream));
}

}  // extern "C"

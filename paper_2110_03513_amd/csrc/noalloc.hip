// noalloc.hip -- cwb_fit_create_noalloc: a fit whose histogram partials live
// in a file-scope device array of the library instead of the caller's
// workspace, for callers that cannot allocate device memory.
//
// The array is reached only through the address hipGetSymbolAddress returns
// for the current device (taken once per device, on the entry point's first
// call there): in host code the array's name is a host-side stand-in, not a
// device address.  Every fit created here on one GPU shares that GPU's
// array, so their runs must not overlap on the device.  Each histogram pass
// writes every word of the partial slots its select pass reads, so nothing
// needs clearing between calls.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/cwb.h"
#include "runtime.h"

namespace cwb {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) long long scratch[kScratchBytes / sizeof(long long)];

std::mutex g_scratch_mu;
long long* g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of the array.
int scratch_for(int dev, long long** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(CWB_E_UNSUPPORTED, "device index above the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(CWB_E_DEVICE, std::string("scratch array address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<long long*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CWB_OK;
}

}  // namespace
}  // namespace cwb

extern "C" int cwb_fit_create_noalloc(const cwb_problem* pr, void* dev_ws, size_t ws_bytes,
                                      void* stream, cwb_fit** out) {
  if (out) *out = nullptr;
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return cwb::set_error(CWB_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  long long* s = nullptr;
  const int rc = cwb::scratch_for(dev, &s);
  if (rc) return rc;
  return cwb::fit_create_with_scratch(pr, dev_ws, ws_bytes, stream, out, s, cwb::kScratchBytes);
}

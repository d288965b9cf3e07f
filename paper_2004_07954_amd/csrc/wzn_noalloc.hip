// wzn_rhs_1d_noalloc: the 1D right-hand side for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).  It runs the kernels of wzn_rhs_1d with
// their scratch (the reduction slot of the Lax-Friedrichs alpha and the debug-scan words) in
// a file-scope device array instead of a caller's workspace.
//
// The array's name is a host-side stand-in in host code; its device address is taken once
// per device with hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels.  Every call on a device shares that device's array: calls that overlap
// on one device (other streams, other host threads) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wzn_host.hpp"

namespace wzn {

static __device__ __align__(256) unsigned long long scratch[WS_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mutex;

// Device address of this device's scratch array, taken on the first call on the device.
static int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return set_error(WZN_ERR_HIP, "wzn_rhs_1d_noalloc: hipGetDevice failed");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return set_error(WZN_ERR_HIP, "wzn_rhs_1d_noalloc: device %d beyond %d", dev,
                     NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(WZN_ERR_HIP, "wzn_rhs_1d_noalloc: hipGetSymbolAddress: %s",
                       hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return WZN_OK;
}

}  // namespace wzn

extern "C" int32_t wzn_rhs_1d_noalloc(const wzn_params* p, const void* u, void* dudt, int64_t n,
                                      double dx, void* stream) {
  void* ws = nullptr;
  const int st = wzn::scratch_address(&ws);
  if (st) return st;
  return wzn_rhs_1d(p, u, dudt, n, dx, ws, stream);
}

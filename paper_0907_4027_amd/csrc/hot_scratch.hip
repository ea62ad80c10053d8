// hot_scratch.hip -- the fixed device workspace of the allocation-free solver entry point
// (hot_gsw_noalloc in hot_api.cpp): one file-scope array, and the lookup of its device address.
#include "hot_internal.h"

#include <mutex>

namespace hot {

// The workspace of hot_gsw_noalloc: the trap tables, the state, the fixed-point trap sums, the
// statistics and the degenerate flag of one call.  Every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` is only a stand-in for the symbol, never a
// device address: the address comes from scratch_address().
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices];
std::mutex g_scratch_mu;
}  // namespace

// Device address of the current device's copy of the workspace; `device` must be the current
// device.  Looked up once per device (hipGetSymbolAddress), then cached.
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace hot

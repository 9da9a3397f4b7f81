// Static device scratch for the allocation-free entry point
// (kp_rmat_apply_noalloc). The array lives in this library's code object; every
// GPU the library runs on holds its own copy, at its own address, from the first
// lookup until the process ends. Host code never passes the array's name to a
// kernel or a copy (on the host that name is only a stand-in): it uses the
// device address that hipGetSymbolAddress returns, looked up once per device
// with that device current (at context creation) and kept here per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "common.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void* g_addr[kMaxDevices] = {};

}  // namespace

namespace kpsb {

size_t scratch_capacity() { return kScratchBytes; }

// Device address of the calling thread's current device's copy of the scratch
// array; looked up on the first call for a device, then cached.
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return e;
    }
    g_addr[device] = p;
  }
  *out = g_addr[device];
  return hipSuccess;
}

}  // namespace kpsb

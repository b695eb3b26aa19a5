// The library's fixed device scratch area, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid allocation): one
// file-scope array per GPU, sized at build time, whose address each device resolves once.
#include <hip/hip_runtime.h>
#include <stddef.h>

#include <mutex>

#include "ifnso_launch.hpp"

namespace ifnso {

// Every GPU the library runs on holds its own copy of this array until the process ends.
// In host code the name stands for a host-side handle, not a device address: kernels and
// copies only ever receive the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch(int device, void **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace ifnso

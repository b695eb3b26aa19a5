// The library's fixed device scratch area, for callers that cannot allocate device memory
// (code under stream capture, tight serving loops, harnesses that forbid allocation): one
// file-scope array per GPU, sized at build time, whose address each device resolves once.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <string.h>

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

// ---------------------------------------------------------------------------------------------
// Small host tables (problem tables of a call) copied to device memory in stream order through
// kernel arguments: the runtime copies a launch's arguments when the launch is enqueued, so the
// host buffer is free again on return and no pinned staging buffer (whose reuse would have to
// wait for the copy) is needed.
// ---------------------------------------------------------------------------------------------
namespace {
constexpr int kUploadWords = 768;  // 3 KiB of arguments per launch
struct UploadChunk {
  uint32_t w[kUploadWords];
};

__global__ __launch_bounds__(256) void k_upload(uint32_t *dst, const UploadChunk c, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += blockDim.x) dst[i] = c.w[i];
}
}  // namespace

hipError_t upload_table(void *dst, const void *src, size_t bytes, hipStream_t s) {
  if (bytes % 4 || (uintptr_t)dst % 4) return hipErrorInvalidValue;
  const uint32_t *w = (const uint32_t *)src;
  const size_t n = bytes / 4;
  UploadChunk c;
  for (size_t o = 0; o < n; o += kUploadWords) {
    const int m = (int)(n - o < (size_t)kUploadWords ? n - o : (size_t)kUploadWords);
    memcpy(c.w, w + o, (size_t)m * 4);
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, (uint32_t *)dst + o, c, m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ifnso

// Copies for request loops: a kernel moves the bytes, reading or writing
// pinned host memory directly over the bus, so the copies of a serving loop
// never wait on the runtime's copy engines.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swih.h"

namespace {

// dst[i] = src[i] for i < n, 16 bytes per thread and step where both
// addresses share their alignment, bytes at the unaligned head and tail.
__global__ __launch_bounds__(256) void k_copy(const unsigned char* __restrict__ src,
                                              unsigned char* __restrict__ dst, size_t n) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t nth = (size_t)gridDim.x * blockDim.x;
  const uintptr_t s = (uintptr_t)src, d = (uintptr_t)dst;
  size_t head = 0, nvec = 0;
  if (((s ^ d) & 15) == 0) {
    head = (16 - (s & 15)) & 15;
    if (head > n) head = n;
    nvec = (n - head) / 16;
  } else {
    head = n;  // no common alignment: bytes only
  }
  for (size_t i = tid; i < head; i += nth) dst[i] = src[i];
  const uint4* __restrict__ s4 = (const uint4*)(src + head);
  uint4* __restrict__ d4 = (uint4*)(dst + head);
  for (size_t i = tid; i < nvec; i += nth) d4[i] = s4[i];
  const size_t tail0 = head + 16 * nvec;
  for (size_t i = tail0 + tid; i < n; i += nth) dst[i] = src[i];
}

// The device address of p: device memory as is, pinned host memory through
// its device mapping; null for memory the device cannot reach.
void* device_view(const void* p) {
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();  // clear the error the lookup of unknown memory leaves
    return nullptr;
  }
  if (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged) return (void*)p;
  if (at.type == hipMemoryTypeHost) return at.devicePointer;
  return nullptr;
}

}  // namespace

extern "C" int swih_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes == 0) return SWIH_OK;
  if (!dst || !src) return SWIH_ERR_INVALID;
  void* dd = device_view(dst);
  const void* ds = device_view(src);
  if (!dd || !ds) return SWIH_ERR_INVALID;
  size_t blocks = (bytes / 16 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     (const unsigned char*)ds, (unsigned char*)dd, bytes);
  return hipGetLastError() == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
}

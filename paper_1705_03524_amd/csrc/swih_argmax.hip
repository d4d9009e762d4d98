// Location of the best window of a likelihood map (the tracker's localisation
// step, Sec. 4): the first maximum in row-major order.
//
// Likelihoods are non-negative floats, whose bit patterns order like their
// values, so key = (bits << 32) | (2^32 - 1 - index) is largest for the
// largest value and, among equal values, for the smallest index.  Each wave
// reduces its keys, then one 64-bit atomic max per wave combines them.
#include "swih.h"
#include "swih_internal.h"
#include "wave64.h"

namespace swih {
namespace {

constexpr int WG = 256;

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }

}  // namespace

__global__ __launch_bounds__(64) void k_argmax_init(uint64_t* key) {
  if (threadIdx.x == 0) key[0] = 0;
}

__global__ __launch_bounds__(WG) void k_argmax(const float* __restrict__ map, int64_t n,
                                               uint64_t* key) {
  uint64_t best = 0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
    const uint32_t bits = __float_as_uint(map[i]);
    best = umax64(best, ((uint64_t)bits << 32) | (uint64_t)(0xffffffffu - (uint32_t)i));
  }
  for (int s = 32; s >= 1; s >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)best, s, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(best >> 32), s, 64);
    best = umax64(best, ((uint64_t)hi << 32) | lo);
  }
  if ((threadIdx.x & 63) == 0) atomicMax((unsigned long long*)key, (unsigned long long)best);
}

}  // namespace swih

extern "C" int swih_argmax(const float* d_map, int64_t n, uint64_t* d_key, void* stream) {
  if (n < 1 || n > 0xffffffffLL || !d_map || !d_key) return SWIH_ERR_INVALID;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(swih::k_argmax_init, dim3(1), dim3(64), 0, s, d_key);
  const int64_t blocks = (n + swih::WG - 1) / swih::WG;
  hipLaunchKernelGGL(swih::k_argmax, dim3((unsigned)(blocks < 2048 ? blocks : 2048)), dim3(swih::WG), 0, s,
                     d_map, n, d_key);
  return hipGetLastError() == hipSuccess ? SWIH_OK : SWIH_ERR_HIP;
}

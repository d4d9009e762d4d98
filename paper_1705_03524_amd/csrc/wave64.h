// Wave64 scan / reduction primitives for gfx950 (CDNA4), built on DPP moves.
//
// Inclusive scan of a 64-lane wave: four row_shr steps (1, 2, 4, 8) give the
// prefix inside each 16-lane row; row_bcast:15 then carries row 0 into row 1
// and row 2 into row 3, and row_bcast:31 carries lanes 0..31 into rows 2-3.
// Disabled or out-of-row source lanes contribute the identity (0).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swih {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += dpp_u32<0x111>(v);         // row_shr:1
  v += dpp_u32<0x112>(v);         // row_shr:2
  v += dpp_u32<0x114>(v);         // row_shr:4
  v += dpp_u32<0x118>(v);         // row_shr:8
  v += dpp_u32<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
  v += dpp_u32<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ __forceinline__ int32_t wave_incl_scan(int32_t v) {
  return (int32_t)wave_incl_scan((uint32_t)v);
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = dpp_u32<CTRL, ROWMASK>((uint32_t)v);
  const uint32_t hi = dpp_u32<CTRL, ROWMASK>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  uint64_t u = (uint64_t)v;
  u += dpp_u64<0x111>(u);
  u += dpp_u64<0x112>(u);
  u += dpp_u64<0x114>(u);
  u += dpp_u64<0x118>(u);
  u += dpp_u64<0x142, 0xa>(u);
  u += dpp_u64<0x143, 0xc>(u);
  return (int64_t)u;
}

template <int CTRL, int ROWMASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  return __builtin_bit_cast(double, dpp_u64<CTRL, ROWMASK>(__builtin_bit_cast(uint64_t, v)));
}

// A disabled lane's DPP result is +0.0 (all-zero bits), the additive identity.
__device__ __forceinline__ double wave_incl_scan(double v) {
  v += dpp_f64<0x111>(v);
  v += dpp_f64<0x112>(v);
  v += dpp_f64<0x114>(v);
  v += dpp_f64<0x118>(v);
  v += dpp_f64<0x142, 0xa>(v);
  v += dpp_f64<0x143, 0xc>(v);
  return v;
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ int32_t readlane(int32_t v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}
__device__ __forceinline__ int64_t readlane(int64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlane(double v, int lane) {
  return __builtin_bit_cast(double, (uint64_t)readlane(__builtin_bit_cast(int64_t, v), lane));
}

// The value v of lane src (src may differ from lane to lane).
__device__ __forceinline__ double lane_value(double v, int src) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Put a wave-uniform value into one lane of a per-lane register.
template <typename T>
__device__ __forceinline__ T put_lane(T reg, T val, int lane) {
  return lane_id() == lane ? val : reg;
}

// 64 x 64 bit transpose across the wave: lane l holds bits A[l][k]; afterwards
// lane k holds A[l][k] at bit l.  Each stage swaps bit s of the lane index with
// bit s of the bit index (the off-diagonal s x s blocks of every 2s x 2s block).
__device__ __forceinline__ uint64_t wave_transpose64(uint64_t m) {
  const int lane = lane_id();
  const uint64_t low[6] = {0x5555555555555555ull, 0x3333333333333333ull, 0x0F0F0F0F0F0F0F0Full,
                           0x00FF00FF00FF00FFull, 0x0000FFFF0000FFFFull, 0x00000000FFFFFFFFull};
#pragma unroll
  for (int b = 5; b >= 0; --b) {
    const int s = 1 << b;
    const uint32_t plo = (uint32_t)__shfl_xor((int)(uint32_t)m, s, 64);
    const uint32_t phi = (uint32_t)__shfl_xor((int)(uint32_t)(m >> 32), s, 64);
    const uint64_t t = ((uint64_t)phi << 32) | plo;
    m = (lane & s) ? (m & ~low[b]) | ((t & ~low[b]) >> s) : (m & low[b]) | ((t & low[b]) << s);
  }
  return m;
}

// Wave total = lane 63 of the inclusive scan.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  return readlane(wave_incl_scan(v), 63);
}

}  // namespace swih

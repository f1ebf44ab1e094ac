// Wavefront (64-lane) primitives for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ks {

constexpr int kWave = 64;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v |= (uint32_t)__shfl_xor((int)v, o);
  return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o);
  return v;
}

// 96-bit sum held as (lo 64, hi 32) with carry propagation.
__device__ __forceinline__ void wave_sum_u96(uint64_t& lo, uint32_t& hi) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t l2 = (uint64_t)__shfl_xor((unsigned long long)lo, o);
    const uint32_t h2 = (uint32_t)__shfl_xor((int)hi, o);
    const uint64_t s = lo + l2;
    hi += h2 + (uint32_t)(s < lo);
    lo = s;
  }
}

// Inclusive prefix sum over the wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t t = (uint32_t)__shfl_up((int)v, o);
    if (l >= (uint32_t)o) v += t;
  }
  return v;
}

}  // namespace ks

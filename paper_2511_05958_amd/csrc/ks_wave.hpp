// Wavefront (64-lane) primitives for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ks {

constexpr int kWave = 64;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Index of the calling wave in its workgroup, marked wave-uniform so that the
// compiler keeps what derives from it (row counters, row geometry, loop
// bounds) in scalar registers and branches with the scalar unit.
__device__ __forceinline__ uint32_t wave_id() {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// ---- DPP reductions (VALU only). After the four in-row steps every lane of a
// 16-lane row holds the row total; row_bcast:15 / row_bcast:31 then fold the
// rows so that lane 63 holds the wave total.
constexpr int kDppXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;
constexpr int kDppMirror = 0x140;
constexpr int kDppBcast15 = 0x142;
constexpr int kDppBcast31 = 0x143;

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, false);
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ void dpp_add96(uint64_t& lo, uint32_t& hi) {
  const uint32_t a = dpp<CTRL, ROW_MASK>((uint32_t)lo);
  const uint32_t b = dpp<CTRL, ROW_MASK>((uint32_t)(lo >> 32));
  const uint32_t c = dpp<CTRL, ROW_MASK>(hi);
  const uint64_t t = ((uint64_t)b << 32) | a;
  const uint64_t s = lo + t;
  hi += c + (uint32_t)(s < lo);
  lo = s;
}

template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ void dpp_add64(uint64_t& v) {
  const uint32_t a = dpp<CTRL, ROW_MASK>((uint32_t)v);
  const uint32_t b = dpp<CTRL, ROW_MASK>((uint32_t)(v >> 32));
  v += ((uint64_t)b << 32) | a;
}

// Wave totals of a 64-bit and a 96-bit sum, returned wave-uniform.
__device__ __forceinline__ void wave_total_64_96(uint64_t& s1, uint64_t& s2, uint32_t& s2h) {
  dpp_add64<kDppXor1>(s1);
  dpp_add96<kDppXor1>(s2, s2h);
  dpp_add64<kDppXor2>(s1);
  dpp_add96<kDppXor2>(s2, s2h);
  dpp_add64<kDppHalfMirror>(s1);
  dpp_add96<kDppHalfMirror>(s2, s2h);
  dpp_add64<kDppMirror>(s1);
  dpp_add96<kDppMirror>(s2, s2h);
  dpp_add64<kDppBcast15, 0xA>(s1);
  dpp_add96<kDppBcast15, 0xA>(s2, s2h);
  dpp_add64<kDppBcast31, 0xC>(s1);
  dpp_add96<kDppBcast31, 0xC>(s2, s2h);
  const uint32_t a = __builtin_amdgcn_readlane((int)(uint32_t)s1, 63);
  const uint32_t b = __builtin_amdgcn_readlane((int)(uint32_t)(s1 >> 32), 63);
  const uint32_t c = __builtin_amdgcn_readlane((int)(uint32_t)s2, 63);
  const uint32_t d = __builtin_amdgcn_readlane((int)(uint32_t)(s2 >> 32), 63);
  s2h = __builtin_amdgcn_readlane((int)s2h, 63);
  s1 = ((uint64_t)b << 32) | a;
  s2 = ((uint64_t)d << 32) | c;
}

// Wave-uniform min / max / or of a 32-bit value (DPP steps, total read from lane 63).
#define KS_DPP_REDUCE32(NAME, OP)                                  \
  __device__ __forceinline__ uint32_t NAME(uint32_t v) {          \
    v = OP(v, dpp<kDppXor1>(v));                                  \
    v = OP(v, dpp<kDppXor2>(v));                                  \
    v = OP(v, dpp<kDppHalfMirror>(v));                            \
    v = OP(v, dpp<kDppMirror>(v));                                \
    v = OP(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, kDppBcast15, 0xA, 0xF, false)); \
    v = OP(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, kDppBcast31, 0xC, 0xF, false)); \
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);     \
  }

__device__ __forceinline__ uint32_t op_min(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t op_max(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t op_or(uint32_t a, uint32_t b) { return a | b; }
KS_DPP_REDUCE32(wave_min_u32, op_min)
KS_DPP_REDUCE32(wave_max_u32, op_max)
KS_DPP_REDUCE32(wave_or_u32, op_or)
#undef KS_DPP_REDUCE32

// Inclusive prefix sum over the wave: shifts by 1, 2, 4, 8 inside each 16-lane
// row (lanes shifted in from outside the row read 0), then the row totals are
// carried forward with row_bcast:15 and row_bcast:31.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppBcast15, 0xA, 0xF, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kDppBcast31, 0xC, 0xF, false);
  return v;
}

}  // namespace ks

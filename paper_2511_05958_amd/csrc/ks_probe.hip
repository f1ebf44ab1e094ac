// Read-bandwidth probe (see include/ks_probe.h).
#include <hip/hip_runtime.h>

#include "ks.h"
#include "ks_ctx.hpp"
#include "ks_probe.h"
#include "ks_wave.hpp"

namespace {

template <int UNROLL>
__global__ __launch_bounds__(256) void probe_read_kernel(const ks::u32x4* __restrict__ p, uint64_t n,
                                                         uint32_t* __restrict__ sink) {
  uint32_t x = 0;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + (UNROLL - 1) * stride < n; i += UNROLL * stride) {
    ks::u32x4 v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n; i += stride) {
    const ks::u32x4 v = __builtin_nontemporal_load(p + i);
    x ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (x == 0x9e3779b9u) sink[0] = x;
}

}  // namespace

extern "C" int ks_probe_read(const uint32_t* words, uint64_t num_words, uint32_t grid, uint32_t unroll,
                             uint32_t* sink, void* stream) {
  if (!words || !sink || grid == 0 || (num_words & 3u) || (reinterpret_cast<uintptr_t>(words) & 15u) ||
      (unroll != 1 && unroll != 8))
    return KS_E_INVALID;
  const ks::u32x4* p = reinterpret_cast<const ks::u32x4*>(words);
  hipStream_t st = (hipStream_t)stream;
  if (unroll == 1)
    hipLaunchKernelGGL(probe_read_kernel<1>, dim3(grid), dim3(256), 0, st, p, num_words / 4, sink);
  else
    hipLaunchKernelGGL(probe_read_kernel<8>, dim3(grid), dim3(256), 0, st, p, num_words / 4, sink);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? KS_OK : ks_host::hip_fail(e, "probe launch");
}

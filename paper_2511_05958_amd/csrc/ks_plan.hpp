// Series order of the row passes: one workgroup buckets the series of a
// batch by row class and sample bytes, so that each class's launch takes its
// own series, longest first. Used by the feature pass and the per-row
// statistics.
#pragma once

#include <hip/hip_runtime.h>

#include "ks.h"
#include "ks_scan.hpp"
#include "ks_select.hpp"

namespace ks {
namespace {  // the kernel is compiled into each translation unit that launches it

// Series order (one workgroup): per row class (1, 2 or 4 load batches,
// streamed, or short rows four to a wave) the series largest first, bucketed
// by the bit length of their sample bytes (a longest-processing-time order,
// so a class's launch starts its longest workgroups first and no workgroup
// waits behind a class it does not belong to); malformed series last in
// class 1.
// plan[0 .. n) is the order, plan[n + c] the first index of class c and
// plan[n + kFeatClasses + c] its count.
constexpr int kFeatPlanNT = 1024;
constexpr uint32_t kFeatBuckets = 40;

constexpr uint32_t kFeatClasses = 5;
__device__ __forceinline__ uint32_t feat_class_index(uint32_t NB) {
  return NB == 1 ? 0u : (NB == 2 ? 1u : (NB == 4 ? 2u : (NB == kStreamed ? 3u : 4u)));
}

__global__ __launch_bounds__(kFeatPlanNT) void feature_plan_kernel(const ks_desc* __restrict__ desc,
                                                                   uint32_t num_series, uint64_t num_samples,
                                                                   uint32_t max_K, uint32_t* __restrict__ plan) {
  __shared__ uint32_t cnt[kFeatClasses * kFeatBuckets];
  const uint32_t tid = threadIdx.x;
  for (uint32_t i = tid; i < kFeatClasses * kFeatBuckets; i += kFeatPlanNT) cnt[i] = 0;
  __syncthreads();
  auto key = [&](uint32_t s) -> uint32_t {
    const ks_desc d = desc[s];
    if (check_desc(d, num_samples, max_K) || d.N > KS_FEATURE_MAX_N) return kFeatBuckets - 1;
    const uint64_t bytes = 4ull * d.K * d.N;  // < 2^38
    const uint32_t bl = 64u - (uint32_t)__clzll(bytes);
    return feat_class_index(feat_batches(d.N)) * kFeatBuckets + (kFeatBuckets - 2 - min(bl, kFeatBuckets - 2));
  };
  for (uint32_t s = tid; s < num_series; s += kFeatPlanNT) atomicAdd(&cnt[key(s)], 1u);
  __syncthreads();
  if (tid == 0) {
    uint32_t run = 0;
    for (uint32_t c = 0; c < kFeatClasses; ++c) {
      plan[num_series + c] = run;
      for (uint32_t b = 0; b < kFeatBuckets; ++b) {
        const uint32_t k = cnt[c * kFeatBuckets + b];
        cnt[c * kFeatBuckets + b] = run;
        run += k;
      }
      plan[num_series + kFeatClasses + c] = run - plan[num_series + c];
    }
  }
  __syncthreads();
  for (uint32_t s = tid; s < num_series; s += kFeatPlanNT) plan[atomicAdd(&cnt[key(s)], 1u)] = s;
}

}  // namespace
}  // namespace ks

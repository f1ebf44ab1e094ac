// Exact refine of a proposal: the full scan's keys, sort, walk and choice,
// with the walk restricted to candidates within +-w of the proposal when its
// confidence reaches tau, over all candidates otherwise (fallback). Reads
// only the per-row moments and series minimum that the proposal pass left in
// the workspace, never the samples.
#pragma once

#include "ks_features.hpp"
#include "ks_scan.hpp"

namespace ks {

template <int KMAX, int NT, int RB>
__global__ __launch_bounds__(NT) void refine_kernel(const ks_desc* __restrict__ desc, uint32_t num_series,
                                                    uint64_t num_samples, uint32_t max_K, ks_params prm,
                                                    const int32_t* __restrict__ proposal,
                                                    const float* __restrict__ confidence, LearnWs lw, uint32_t SR,
                                                    ks_result* __restrict__ out) {
  __shared__ ScanSmem<KMAX, NT, RB> sm;
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  uint32_t bad = check_desc(d, num_samples, max_K);
  if (!bad && lw.K[s] != d.K) bad = KS_BAD_SHAPE;  // the proposal pass skipped this series
  if (bad) {
    if (threadIdx.x == 0) write_result(out + s, 0, 0, 0, 0, 0.0, 0.0, 1.0, bad);
    return;
  }
  const uint32_t K = d.K;
  const uint64_t slot = (uint64_t)s * SR + 2;
  for (uint32_t i = threadIdx.x; i < K; i += NT) {
    sm.u.mom.s1[i] = lw.s1[slot + i];
    sm.u.mom.s2lo[i] = lw.s2lo[slot + i];
    sm.u.mom.s2hi[i] = lw.s2hi[slot + i];
  }
  const uint32_t gmin = lw.smin[s];
  __syncthreads();
  const int64_t p = proposal[s];
  const float cf = confidence[s];
  bool refined = cf >= prm.tau;  // NaN confidence falls back
  int64_t lo = p - (int64_t)prm.w, hi = p + (int64_t)prm.w;
  if (lo < 1) lo = 1;
  if (hi > (int64_t)K - 1) hi = (int64_t)K - 1;
  if (lo > hi) refined = false;
  if (!refined) {
    lo = 1;
    hi = (int64_t)K - 1;
  }
  finish_series(sm, K, d.N, gmin, prm, out + s, nullptr, (uint32_t)lo, (uint32_t)hi,
                refined ? KS_REFINED : KS_FALLBACK);
}

}  // namespace ks

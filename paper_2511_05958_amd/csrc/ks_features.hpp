// Learned-proposal stage 1: one read of every sample gives, per row,
//   - the moments (sum r, sum r^2) that the exact refine turns into eq. 2 keys,
//   - the nine deciles x_(floor(k (N-1) / 10)), k = 1..9, by a wave-level
//     radix select over the row's uint32 cycle counts (keys r - row minimum,
//     as many digit levels as the row's range needs),
// and per series the minimum m, then features f = (double)(x - m) / max(m, 1)
// rounded to float (project-defined inputs of the network).
#pragma once

#include "ks_cnn.hpp"
#include "ks_scan.hpp"
#include "ks_select.hpp"

namespace ks {

// Per-row moments of the learned path (the refine's input), per-series min.
struct LearnWs {
  uint64_t* s1;     // [num_series * SR] (row slot of series s: s * SR + 2 + i)
  uint64_t* s2lo;
  uint32_t* s2hi;
  uint32_t* smin;   // [num_series]
  uint32_t* K;      // [num_series]: K when the series was valid, 0 otherwise
};

// Features of one series per workgroup (series whose rows need NB batches;
// the NB = 1 launch also clears the slots of malformed series). One wave per
// row, rows w, w + 4, ... for wave w. Writes: the caller's FP32 features
// (nullable, rows at aux_offset), the network input rows (bf16, 16 channels,
// 11 used) at row slot s * SR + 2 + i, and the refine workspace.
template <int NB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NB == 4 ? 3 : 1))) void features_kernel(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                      const ks_desc* __restrict__ desc, uint32_t num_series,
                                                      uint32_t max_K, float* __restrict__ feat_out,
                                                      uint64_t feat_rows, uint16_t* __restrict__ x0,
                                                      uint32_t SR, LearnWs lw, float* __restrict__ feat_ws) {
  constexpr int W = NT / kWave;
  __shared__ SelLds sel[W];
  __shared__ uint32_t red[W];
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const uint32_t tid = threadIdx.x, lane = lane_id();
  const uint32_t w = wave_id();
  const bool bad = check_desc(d, num_samples, max_K) || d.N > KS_FEATURE_MAX_N;
  if ((bad ? 1u : feat_batches(d.N)) != (uint32_t)NB) return;
  if (bad) {
    for (uint32_t q = tid; q < SR * 16; q += NT) x0[(uint64_t)s * SR * 16 + q] = 0;
    if (tid == 0) lw.K[s] = 0;
    return;
  }
  const uint32_t K = d.K, N = d.N;
  const uint64_t slot = (uint64_t)s * SR + 2;
  SelLds& L = sel[w];
  uint32_t gmin = 0xffffffffu;
  Batch cur[NB];
  RowGeo g;
  if (w < K) g = load_row<NB>(cur, samples, d.offset + (uint64_t)w * N, N, lane);
  for (uint32_t i = w; i < K; i += W) {
    uint64_t s1, s2;
    uint32_t s2h;
    const RowScan rs = row_scan<NB>(L, cur, g, N, s1, s2, s2h, lane);
    // the next row's loads are in flight while this row's order statistics are found
    const RowGeo gi = g;
    if (i + W < K) g = load_row<NB>(cur, samples, d.offset + (uint64_t)(i + W) * N, N, lane);
    if (lane == 0) {
      lw.s1[slot + i] = s1;
      lw.s2lo[slot + i] = s2;
      lw.s2hi[slot + i] = s2h;
    }
    const uint32_t dec = row_select<NB, DecileRanks>(L, samples, gi, rs, N, lane);
    gmin = min(gmin, rs.rmin);
    // feature numerators x - m need the series minimum: keep x itself
    if (lane < 9) feat_ws[(slot + i) * 9 + lane] = __uint_as_float(dec);
  }
  if (lane == 0) red[w] = gmin;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < W; ++u) gmin = min(gmin, red[u]);
  // second sweep: normalise by the series minimum
  const double denom = (double)(gmin > 1 ? gmin : 1u);
  const bool to_user = feat_out && d.aux_offset <= feat_rows && K <= feat_rows - d.aux_offset;
  for (uint32_t q = tid; q < K * 9; q += NT) {
    const uint32_t i = q / 9, k = q - i * 9;
    const uint32_t x = __float_as_uint(feat_ws[(slot + i) * 9 + k]);
    const float f = (float)((double)(x - gmin) / denom);
    feat_ws[(slot + i) * 9 + k] = f;
    if (to_user) feat_out[(d.aux_offset + i) * 9 + k] = f;
  }
  __syncthreads();
  // network input: bf16 of the features and the two position channels, 16
  // channels per row (11..15 zero); the slot's rows outside [2, 2 + K) stay
  // zero (they are the conv's zero padding)
  const uint64_t base = (uint64_t)s * SR;
  for (uint32_t q = tid; q < SR * 16; q += NT) {
    const uint32_t r = q / 16, k = q - r * 16;
    uint16_t b = 0;
    if (r >= 2 && r < K + 2) {
      if (k < 9)
        b = cnn::f2bf(feat_ws[(base + r) * 9 + k]);
      else if (k == 9)
        b = cnn::f2bf(cnn::pos_frac(r - 2, K));
      else if (k == 10)
        b = cnn::f2bf(cnn::pos_centre(r - 2, K));
    }
    x0[(base + r) * 16 + k] = b;
  }
  if (tid == 0) {
    lw.smin[s] = gmin;
    lw.K[s] = K;
  }
}

}  // namespace ks

// Learned-proposal stage 1: one read of every sample gives, per row,
//   - the moments (sum r, sum r^2) that the exact refine turns into eq. 2 keys,
//   - the nine deciles x_(floor(k (N-1) / 10)), k = 1..9, by the wave-level
//     select of ks_select.hpp (a 1024-bin window of the keys above the row's
//     minimum or a base just below it, radix levels only past the window),
// and per series the minimum m, then features f = (double)(x - m) / max(m, 1)
// rounded to float (project-defined inputs of the network).
#pragma once

#include "ks_cnn.hpp"
#include "ks_scan.hpp"
#include "ks_plan.hpp"
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

// Per-wave staging of a wave's per-row outputs: a wave takes a contiguous
// block of rows and writes every kFeatStage rows' deciles and moments as
// contiguous stores (rows written one at a time, by waves interleaved row by
// row, left partly written cache lines behind; they cost 5 - 15% of the
// pass and made its time depend on where the buffers lay in memory). Rows of
// two or more load batches stage 64 rows (fewer, longer write bursts among
// the reads: the learned step on 8192 x 1024 x 2048 ran 1 - 4% faster than
// with 16); one-batch and short rows stage 16, which keeps their LDS within
// six workgroups per CU.
// (at most 64: a flush writes one row's moments per lane)
__host__ __device__ constexpr uint32_t feat_stage_rows(int NB) { return NB == 1 || NB == (int)kGrouped ? 16u : 64u; }

template <uint32_t S>
struct FeatStage {
  uint32_t dec[S * 9];
  uint64_t s1[S], s2lo[S];
  uint32_t s2hi[S];
};

// First step, workgroup t of the launch of row class NB (rows in 1, 2 or 4
// load batches held in registers, kStreamed, or kGrouped) takes the t-th
// series of that class in the plan's order (the NB = 1 launch also marks
// malformed series with K = 0). One wave per row (four per step for kGrouped);
// wave w of W takes rows [w B, (w + 1) B) with B = ceil(K / W). Writes per row
// the deciles (as raw samples, at row slot s * SR + 2 + i of feat_ws) and the
// refine workspace's moments, and per series its minimum and K.
template <int NB, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(feat_waves_per_eu(NB)))) void features_kernel(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                      const ks_desc* __restrict__ desc, uint32_t num_series,
                                                      uint32_t max_K, uint32_t SR, LearnWs lw,
                                                      float* __restrict__ feat_ws,
                                                      const uint32_t* __restrict__ plan) {
  constexpr int W = NT / kWave;
  __shared__ RowLds sel[W];
  constexpr uint32_t kFeatStage = feat_stage_rows(NB);
  static_assert(kFeatStage <= (uint32_t)kWave, "a flush writes one row's moments per lane");
  __shared__ FeatStage<kFeatStage> stage[W];
  __shared__ uint32_t red[W];
  const uint32_t ci = feat_class_index(NB);
  if (blockIdx.x >= plan[num_series + kFeatClasses + ci]) return;
  const uint32_t s = plan[plan[num_series + ci] + blockIdx.x];
  const ks_desc d = desc[s];
  const uint32_t tid = threadIdx.x, lane = lane_id();
  const uint32_t w = wave_id();
  const bool bad = check_desc(d, num_samples, max_K) || d.N > KS_FEATURE_MAX_N;
  if ((bad ? 1u : feat_batches(d.N)) != (uint32_t)NB) return;
  if (bad) {  // the pack step zeroes its network input rows
    if (tid == 0) lw.K[s] = 0;
    return;
  }
  const uint32_t K = d.K, N = d.N;
  const uint64_t slot = (uint64_t)s * SR + 2;
  RowLds& L = sel[w];
  FeatStage<kFeatStage>& st = stage[w];
  const uint32_t B = (K + W - 1) / W;
  const uint32_t begin = min(w * B, K), end = min(begin + B, K);
  uint32_t gmin = 0xffffffffu;
  // row i's results; its deciles on lanes first .. first + 8
  auto emit = [&](uint32_t i, uint64_t s1, uint64_t s2, uint32_t s2h, uint32_t rmin, uint32_t dec, uint32_t first) {
    const uint32_t j = (i - begin) % kFeatStage;
    if (lane == 0) {
      st.s1[j] = s1;
      st.s2lo[j] = s2;
      st.s2hi[j] = s2h;
    }
    gmin = min(gmin, rmin);
    // feature numerators x - m need the series minimum: keep x itself
    if (lane - first < 9u) st.dec[j * 9 + lane - first] = dec;
    if (j + 1 == kFeatStage || i + 1 == end) {  // flush rows i - j .. i
      wave_lds_sync();
      const uint64_t r0 = slot + i - j;
      for (uint32_t q = lane; q < (j + 1) * 9; q += kWave)
        row_out_store<NB>(__uint_as_float(st.dec[q]), &feat_ws[r0 * 9 + q]);
      if (lane <= j) {
        row_out_store<NB>(st.s1[lane], &lw.s1[r0 + lane]);
        row_out_store<NB>(st.s2lo[lane], &lw.s2lo[r0 + lane]);
        row_out_store<NB>(st.s2hi[lane], &lw.s2hi[r0 + lane]);
      }
      wave_lds_sync();
    }
  };
  if constexpr (NB == (int)kStreamed) {
    select_rows_long<DecileRanks>(L, samples, d.offset, N, end, begin, 1u, lane,
                                  [&](uint32_t i, const RowOut& o) { emit(i, o.s1, o.s2, o.s2h, o.rmin, o.sel, 0u); });
  } else if constexpr (NB == (int)kGrouped) {
    select_rows_grouped<DecileRanks>(L, samples, d.offset, N, begin, end, lane,
                                     [&](uint32_t i, const RowOut& o, uint32_t first) {
                                       emit(i, o.s1, o.s2, o.s2h, o.rmin, o.sel, first);
                                     });
  } else {
    Batch cur[NB];
    RowGeo g;
    if (begin < end) g = load_row<NB>(cur, samples, d.offset + (uint64_t)begin * N, N, lane);
    uint32_t p = 0;  // window base from the previous row (none for the first)
    for (uint32_t i = begin; i < end; ++i) {
      uint64_t s1, s2;
      uint32_t s2h;
      RowScan rs;
      const bool based = i > begin && row_scan_based<NB>(L, cur, g, N, p, s1, s2, s2h, rs, lane);
      if (!based) rs = row_scan<NB>(L, cur, g, N, s1, s2, s2h, lane);
      // the next row's loads are in flight while this row's order statistics are found
      const RowGeo gi = g;
      if (i + 1 < end) g = load_row<NB>(cur, samples, d.offset + (uint64_t)(i + 1) * N, N, lane);
      const uint32_t sel = based ? select_from_window<DecileRanks>(L, samples, gi, p, rs.rmax, N, lane)
                                 : row_select<NB, DecileRanks>(L, samples, gi, rs, N, lane);
      p = rs.rmin > kRowMargin ? rs.rmin - kRowMargin : 0u;
      emit(i, s1, s2, s2h, rs.rmin, sel, 0u);
    }
  }
  if (lane == 0) red[w] = gmin;
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int u = 0; u < W; ++u) gmin = min(gmin, red[u]);
    lw.smin[s] = gmin;
    lw.K[s] = K;
  }
}

// Second step, one workgroup per (series, chunk of NT slot rows): the deciles
// x of the series' rows become the features f = (double)(x - m) / max(m, 1)
// rounded to float (m the series minimum), in place and into the caller's
// buffer, element by element (consecutive threads, consecutive elements);
// then the chunk's network input rows (bf16 of the nine features and the two
// position channels, channels 11..15 zero), staged in LDS, are written as
// 16-byte stores. The two slot rows on each side of [2, 2 + K) (the
// convolutions' zero padding) and the first four rows of a malformed series
// (K = 0) are zero; a chunk wholly past row K + 4 writes nothing, as no
// output row of the network reads its inputs there.
template <int NT>
__global__ __launch_bounds__(NT) void feature_pack_kernel(const ks_desc* __restrict__ desc, uint32_t num_series,
                                                          float* __restrict__ feat_out, uint64_t feat_rows,
                                                          uint16_t* __restrict__ x0, uint32_t SR, LearnWs lw,
                                                          float* __restrict__ feat_ws) {
  __shared__ __align__(16) uint16_t bf[NT * 16];
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const uint32_t tid = threadIdx.x;
  const uint32_t r0 = blockIdx.y * NT;
  if (r0 >= SR) return;
  const uint32_t nr = SR - r0 < (uint32_t)NT ? SR - r0 : (uint32_t)NT;
  const uint32_t K = lw.K[s];
  if (r0 >= K + 4u) return;
  const uint64_t row0 = (uint64_t)s * SR + r0;
  // rows [lo, hi) of the chunk hold data
  const uint32_t lo = r0 < 2u ? 2u - r0 : 0u;
  const uint32_t hi = K + 2u > r0 ? (K + 2u - r0 < nr ? K + 2u - r0 : nr) : 0u;
  if (lo < hi) {
    const uint32_t gmin = lw.smin[s];
    const double denom = (double)(gmin > 1 ? gmin : 1u);
    const ks_desc d = desc[s];
    const bool to_user = feat_out && d.aux_offset <= feat_rows && K <= feat_rows - d.aux_offset;
    for (uint32_t q = lo * 9u + tid; q < hi * 9u; q += NT) {
      const uint32_t rr = q / 9u, k = q - rr * 9u;
      const uint64_t e = row0 * 9u + q;
      const uint32_t x = __float_as_uint(feat_ws[e]);
      const float f = (float)((double)(x - gmin) / denom);
      feat_ws[e] = f;
      if (to_user) feat_out[(d.aux_offset + r0 + rr - 2) * 9 + k] = f;
      bf[rr * 16 + k] = cnn::f2bf(f);
    }
  }
  __syncthreads();
  for (uint32_t q = tid; q < nr * 2u; q += NT) {
    const uint32_t rr = q >> 1, h = q & 1u;
    u32x4 v{0u, 0u, 0u, 0u};
    if (rr >= lo && rr < hi) {
      const uint32_t t = r0 + rr - 2;
      if (h == 0) {
        const u32x4 a = *reinterpret_cast<const u32x4*>(&bf[rr * 16]);
        v = a;
      } else {
        const uint32_t b8 = bf[rr * 16 + 8];
        const uint32_t p9 = cnn::f2bf(cnn::pos_frac(t, K)), p10 = cnn::f2bf(cnn::pos_centre(t, K));
        v = u32x4{b8 | (p9 << 16), p10, 0u, 0u};
      }
    }
    *reinterpret_cast<u32x4*>(x0 + (row0 + rr) * 16 + h * 8) = v;
  }
}

}  // namespace ks

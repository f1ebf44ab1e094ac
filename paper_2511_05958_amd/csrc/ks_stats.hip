// Per-row latency statistics (ks_stats_batch): the average as the main result,
// with p50, p95, standard deviation, minimum and maximum beside it, for every
// row of every series in one read of the samples. One wave per row, the row
// in registers; the two percentiles come from the same multi-rank radix
// select as the learned path's deciles.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ks.h"
#include "ks_ctx.hpp"
#include "ks_plan.hpp"
#include "ks_scan.hpp"
#include "ks_select.hpp"

static_assert(sizeof(ks_desc) == 24 && sizeof(ks_result) == 48 && sizeof(ks_params) == 32 &&
                  sizeof(ks_row_stats) == 32,
              "ABI struct sizes");

using namespace ks_host;

namespace {

// p50 and p95: x_(floor(q (N - 1))) for q = 0.5, 0.95.
struct StatRanks {
  static constexpr uint32_t kCount = 2;
  __device__ static uint32_t rank(uint32_t j, uint32_t N) {
    return j == 0 ? (N - 1) / 2u : (uint32_t)((95ull * (N - 1)) / 100u);
  }
};

typedef unsigned __int128 u128;

// u128 -> double, rounded to nearest even once: the top 64 significant bits
// with a sticky bit for everything below, converted, then scaled exactly.
__device__ double u128_to_double(u128 v) {
  const uint64_t hi = (uint64_t)(v >> 64);
  if (hi == 0) return (double)(uint64_t)v;
  const int sh = 64 - __clzll(hi);  // bits above the low 64
  const uint64_t top = (uint64_t)(v >> sh);
  const bool sticky = (v & (((u128)1 << sh) - 1)) != 0;
  return ldexp((double)(top | (uint64_t)sticky), sh);
}

template <int NB>
__global__ __launch_bounds__(ks::row_pass_threads(NB)) __attribute__((amdgpu_waves_per_eu(ks::stats_waves_per_eu(NB)))) void row_stats_kernel(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                        const ks_desc* __restrict__ desc, uint32_t num_series,
                                                        uint32_t max_K, ks_row_stats* __restrict__ out,
                                                        uint64_t out_rows, const uint32_t* __restrict__ plan) {
  constexpr int W = ks::row_pass_threads(NB) / ks::kWave;
  // rows per contiguous write of a wave's records (64 for rows of two or more
  // load batches: fewer, longer write bursts among the reads)
  constexpr uint32_t kStage = NB == 1 || NB == (int)ks::kGrouped ? 16u : 64u;
  static_assert(kStage <= (uint32_t)ks::kWave, "a flush makes one record per lane");
  // a row's exact results, staged until kStage rows are done; the records
  // (mean, std in FP64) are then made by kStage lanes at once
  struct RowStage {
    uint64_t s1[kStage], s2[kStage];
    uint32_t s2h[kStage], rmin[kStage], rmax[kStage], p50[kStage], p95[kStage];
  };
  __shared__ ks::RowLds sel[W];
  __shared__ RowStage stage[W];
  // workgroup t takes the t-th series of this row class in the plan's order
  // (largest first; malformed series in class 1)
  const uint32_t ci = ks::feat_class_index(NB);
  if (blockIdx.x >= plan[num_series + ks::kFeatClasses + ci]) return;
  const uint32_t s = plan[plan[num_series + ci] + blockIdx.x];
  const ks_desc d = desc[s];
  const uint32_t lane = ks::lane_id(), w = ks::wave_id();
  const bool bad = ks::check_desc(d, num_samples, max_K) || d.N > KS_FEATURE_MAX_N;
  if ((bad ? 1u : ks::feat_batches(d.N)) != (uint32_t)NB) return;
  const bool fits = d.aux_offset <= out_rows && (uint64_t)d.K <= out_rows - d.aux_offset;
  if (!fits) return;
  ks_row_stats* o = out + d.aux_offset;
  if (bad) {
    for (uint32_t i = threadIdx.x; i < d.K; i += (uint32_t)ks::row_pass_threads(NB)) o[i] = ks_row_stats{NAN, NAN, 0u, 0u, 0u, 0u};
    return;
  }
  const uint32_t K = d.K, N = d.N;
  ks::RowLds& L = sel[w];
  // wave w takes rows [w B, (w + 1) B) and writes every kStage rows' records as
  // contiguous 16-byte stores (records written one at a time, by waves
  // interleaved row by row, left partly written cache lines behind)
  const uint32_t B = (K + W - 1) / W;
  const uint32_t begin = min(w * B, K), end = min(begin + B, K);
  RowStage& st = stage[w];
  // row i's results; its p50 and p95 on lanes first and first + 1 of sel_x
  auto emit = [&](uint32_t i, uint64_t s1, uint64_t s2, uint32_t s2h, uint32_t rmin, uint32_t rmax, uint32_t sel_x,
                  uint32_t first) {
    const uint32_t p50 = (uint32_t)__builtin_amdgcn_readlane((int)sel_x, (int)first);
    const uint32_t p95 = (uint32_t)__builtin_amdgcn_readlane((int)sel_x, (int)first + 1);
    const uint32_t j = (i - begin) % kStage;
    if (lane == 0) {
      st.s1[j] = s1;
      st.s2[j] = s2;
      st.s2h[j] = s2h;
      st.rmin[j] = rmin;
      st.rmax[j] = rmax;
      st.p50[j] = p50;
      st.p95[j] = p95;
    }
    if (j + 1 == kStage || i + 1 == end) {  // rows i - j .. i: lane q makes row i - j + q's record
      ks::wave_lds_sync();
      if (lane <= j) {
        const uint64_t a1 = st.s1[lane];
        const u128 S2 = ((u128)st.s2h[lane] << 64) | st.s2[lane];
        const u128 num = (u128)N * S2 - (u128)a1 * a1;  // >= 0 (Cauchy-Schwarz), < 2^113
        const double nn = (double)N * (double)N;
        const ks_row_stats r{(double)a1 / (double)N, sqrt(u128_to_double(num) / nn), st.rmin[lane], st.p50[lane],
                             st.p95[lane], st.rmax[lane]};
        static_assert(sizeof(ks_row_stats) == 32, "a record is two 16-byte stores");
        ks::u32x4 v0, v1;
        __builtin_memcpy(&v0, &r, 16);
        __builtin_memcpy(&v1, reinterpret_cast<const char*>(&r) + 16, 16);
        ks::u32x4* dst = reinterpret_cast<ks::u32x4*>(o + (i - j) + lane);
        ks::row_out_store<NB>(v0, dst);
        ks::row_out_store<NB>(v1, dst + 1);
      }
      ks::wave_lds_sync();
    }
  };
  if constexpr (NB == (int)ks::kStreamed) {
    ks::select_rows_long<StatRanks>(L, samples, d.offset, N, end, begin, 1u, lane, [&](uint32_t i, const ks::RowOut& r) {
      emit(i, r.s1, r.s2, r.s2h, r.rmin, r.rmax, r.sel, 0u);
    });
  } else if constexpr (NB == (int)ks::kGrouped) {
    ks::select_rows_grouped<StatRanks>(L, samples, d.offset, N, begin, end, lane,
                                       [&](uint32_t i, const ks::RowOut& r, uint32_t first) {
                                         emit(i, r.s1, r.s2, r.s2h, r.rmin, r.rmax, r.sel, first);
                                       });
  } else {
    ks::Batch cur[NB];
    ks::RowGeo g;
    if (begin < end) g = ks::load_row<NB>(cur, samples, d.offset + (uint64_t)begin * N, N, lane);
    uint32_t p = 0;  // window base from the previous row (none for the first)
    for (uint32_t i = begin; i < end; ++i) {
      uint64_t s1, s2;
      uint32_t s2h;
      ks::RowScan rs;
      const bool based = i > begin && ks::row_scan_based<NB>(L, cur, g, N, p, s1, s2, s2h, rs, lane);
      if (!based) rs = ks::row_scan<NB>(L, cur, g, N, s1, s2, s2h, lane);
      // the next row's loads are in flight while this row's percentiles are found
      const ks::RowGeo gi = g;
      if (i + 1 < end) g = ks::load_row<NB>(cur, samples, d.offset + (uint64_t)(i + 1) * N, N, lane);
      const uint32_t sel = based ? ks::select_from_window<StatRanks>(L, samples, gi, p, rs.rmax, N, lane)
                                 : ks::row_select<NB, StatRanks>(L, samples, gi, rs, N, lane);
      p = rs.rmin > ks::kRowMargin ? rs.rmin - ks::kRowMargin : 0u;
      emit(i, s1, s2, s2h, rs.rmin, rs.rmax, sel, 0u);
    }
  }
}

}  // namespace

extern "C" int ks_stats_batch(ks_ctx* ctx, const uint32_t* samples, uint64_t num_samples, const ks_desc* desc,
                              uint32_t num_series, uint32_t max_K, ks_row_stats* out, uint64_t out_rows, void* stream) {
  if (!ctx) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (max_K < 2 || max_K > KS_MAX_K) return KS_E_RANGE;
  if (num_series == 0) return KS_OK;
  if (!samples || !desc || !out) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  // the series order per row class (the feature pass's plan), kept in the
  // context's scan workspace (its queue items: 512 bytes per series); then one
  // launch per row class (1, 2 or 4 load batches per row, streamed, or short
  // rows four to a wave), each taking its own series largest first
  if (int rc = ks_reserve(ctx, num_series, 0)) return rc;
  uint32_t* plan = reinterpret_cast<uint32_t*>(ctx->items);
  hipLaunchKernelGGL(ks::feature_plan_kernel, dim3(1), dim3(ks::kFeatPlanNT), 0, st, desc, num_series, num_samples,
                     max_K, plan);
  hipLaunchKernelGGL(row_stats_kernel<1>, dim3(num_series), dim3(ks::row_pass_threads(1)), 0, st, samples, num_samples, desc, num_series,
                     max_K, out, out_rows, (const uint32_t*)plan);
  hipLaunchKernelGGL(row_stats_kernel<2>, dim3(num_series), dim3(ks::row_pass_threads(2)), 0, st, samples, num_samples, desc, num_series,
                     max_K, out, out_rows, (const uint32_t*)plan);
  hipLaunchKernelGGL(row_stats_kernel<4>, dim3(num_series), dim3(ks::row_pass_threads(4)), 0, st, samples, num_samples, desc, num_series,
                     max_K, out, out_rows, (const uint32_t*)plan);
  hipLaunchKernelGGL(row_stats_kernel<ks::kStreamed>, dim3(num_series), dim3(ks::row_pass_threads(ks::kStreamed)), 0, st, samples, num_samples, desc,
                     num_series, max_K, out, out_rows, (const uint32_t*)plan);
  hipLaunchKernelGGL(row_stats_kernel<ks::kGrouped>, dim3(num_series), dim3(ks::row_pass_threads(ks::kGrouped)), 0, st, samples, num_samples, desc,
                     num_series, max_K, out, out_rows, (const uint32_t*)plan);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "row stats launch");
}

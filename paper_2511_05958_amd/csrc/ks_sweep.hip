// What the measurement workflow does around one detection: the outlier check
// and interval widening of workflow step 3 (ks_check_batch), the L2 segment
// alignment (ks_align_batch) and the cache-line-size scoring (ks_line_batch).
// All three run on results already on the device (ks_result, ks_row_stats);
// the reading of each rule is stated in include/ks_sweep.h.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ks.h"
#include "ks_ctx.hpp"
#include "ks_scan.hpp"
#include "ks_select.hpp"
#include "ks_sweep.h"

static_assert(sizeof(ks_check) == 32 && sizeof(ks_line) == 24 && sizeof(ks_row_stats) == 32, "ABI struct sizes");

using namespace ks_host;

namespace {

typedef unsigned __int128 u128;

constexpr int kCheckV = 32;  // steps per lane: K <= 64 * 32 = KS_MAX_K
constexpr uint32_t kLineMaxJ = 64, kLineMaxA = 256;

// Lower median x_(floor((n - 1) / 2)).
struct MedianRank {
  static constexpr uint32_t kCount = 1;
  __device__ static uint32_t rank(uint32_t, uint32_t N) { return (N - 1) / 2; }
};

// Lower median of the values v[e] (step lane + 64 e) whose bit e of `in` is
// set, n >= 1 of them over the wave; wave-uniform.
__device__ uint32_t lower_median(ks::SelLds& L, const uint32_t (&v)[kCheckV], uint32_t in, uint32_t n,
                                 uint32_t lane) {
  uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
  for (int e = 0; e < kCheckV; ++e)
    if ((in >> e) & 1u) {
      mn = min(mn, v[e]);
      mx = max(mx, v[e]);
    }
  mn = ks::wave_min_u32(mn);
  mx = ks::wave_max_u32(mx);
  if (mx == mn) return mn;
  const uint32_t b = 32u - __clz(mx - mn);
  uint32_t k[kCheckV];
#pragma unroll
  for (int e = 0; e < kCheckV; ++e) k[e] = ((in >> e) & 1u) ? v[e] - mn : 0xffffffffu;
  const uint32_t key = ks::wave_select<kCheckV, MedianRank>(L, k, b, n, lane);
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)key) + mn;  // lane 0 holds the median's key
}

// Level (median), spread (MAD) and disturbed-step count of the steps [a, b).
__device__ void side_check(ks::SelLds& L, const uint32_t (&v)[kCheckV], uint32_t a, uint32_t b, uint32_t k,
                           uint32_t lane, uint32_t& med, uint32_t& mad, uint32_t& disturbed) {
  uint32_t in = 0;
#pragma unroll
  for (int e = 0; e < kCheckV; ++e) {
    const uint32_t i = lane + ks::kWave * (uint32_t)e;
    in |= (i >= a && i < b) ? 1u << e : 0u;
  }
  const uint32_t n = b - a;
  med = lower_median(L, v, in, n, lane);
  uint32_t dev[kCheckV];
#pragma unroll
  for (int e = 0; e < kCheckV; ++e) dev[e] = v[e] > med ? v[e] - med : med - v[e];
  mad = lower_median(L, dev, in, n, lane);
  const uint64_t thr = (uint64_t)k * max(mad, max(1u, med / 64u));
  uint32_t cnt = 0;
#pragma unroll
  for (int e = 0; e < kCheckV; ++e) cnt += (uint32_t)__popcll(ks::ballot(((in >> e) & 1u) && dev[e] > thr));
  disturbed = cnt;
}

// One wave per sweep, four per workgroup.
__global__ __launch_bounds__(256) void check_kernel(const ks_desc* __restrict__ desc, uint32_t num_series,
                                                    uint32_t max_K, const ks_result* __restrict__ res,
                                                    const ks_row_stats* __restrict__ stats, uint64_t stats_rows,
                                                    uint32_t edge, uint32_t k, ks_check* __restrict__ out) {
  __shared__ ks::SelLds sel[4];
  const uint32_t lane = ks::lane_id(), w = ks::wave_id();
  const uint32_t s = blockIdx.x * 4u + w;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const ks_result r = res[s];
  const uint32_t K = d.K;
  const bool bad = K < 2 || K > max_K || (r.flags & (KS_BAD_SHAPE | KS_OUT_OF_RANGE)) != 0 ||
                   d.aux_offset > stats_rows || (uint64_t)K > stats_rows - d.aux_offset ||
                   ((r.flags & KS_SIGNIFICANT) && (r.cp < 1 || r.cp >= K));
  if (bad) {
    if (lane == 0) out[s] = ks_check{KS_CHECK_INVALID, 0u, 0, 0, 0u, 0u, 0u, 0u};
    return;
  }
  uint32_t v[kCheckV];
#pragma unroll
  for (int e = 0; e < kCheckV; ++e) {
    const uint32_t i = lane + ks::kWave * (uint32_t)e;
    v[e] = i < K ? stats[d.aux_offset + i].p50 : 0u;
  }
  ks::SelLds& L = sel[w];
  const bool sig = (r.flags & KS_SIGNIFICANT) != 0;
  uint32_t med_lo, mad_lo, n_lo, med_hi, mad_hi, n_hi;
  if (sig) {
    side_check(L, v, 0, r.cp, k, lane, med_lo, mad_lo, n_lo);
    side_check(L, v, r.cp, K, k, lane, med_hi, mad_hi, n_hi);
  } else {
    side_check(L, v, 0, K, k, lane, med_lo, mad_lo, n_lo);
    med_hi = med_lo;
    mad_hi = mad_lo;
    n_hi = 0;
  }
  uint32_t flags = 0;
  int32_t lo = 0, hi = (int32_t)K;
  if (!sig) {
    flags |= KS_CHECK_NO_CHANGE;
    lo = -(int32_t)K;
    hi = 2 * (int32_t)K;
  } else {
    if (r.cp < edge) {
      flags |= KS_CHECK_EDGE_LOW;
      lo = -(int32_t)K;
    }
    if (K - r.cp < edge) {
      flags |= KS_CHECK_EDGE_HIGH;
      hi = 2 * (int32_t)K;
    }
  }
  const uint32_t disturbed = n_lo + n_hi;
  if (disturbed) {
    flags |= KS_CHECK_DISTURBED;
    lo = min(lo, -(int32_t)(K / 2));
    hi = max(hi, (int32_t)(K + K / 2));
  }
  if (lane == 0) out[s] = ks_check{flags, disturbed, lo, hi, med_lo, med_hi, mad_lo, mad_hi};
}

// One thread per item: the nearest of T / k, k = floor(T / S) - 1 .. + 2
// (k >= 1), distances |S - T / k| = |S k - T| / k compared exactly.
__global__ __launch_bounds__(256) void align_kernel(const uint64_t* __restrict__ measured,
                                                    const uint64_t* __restrict__ total, uint32_t n,
                                                    uint32_t* __restrict__ segments, double* __restrict__ aligned,
                                                    double* __restrict__ distance) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= n) return;
  const uint64_t S = measured[i], T = total[i];
  constexpr uint64_t kLim = 1ull << 50;
  if (S < 1 || T < 1 || S >= kLim || T >= kLim || T / S > 0xfffffff0ull) {
    segments[i] = 0;
    aligned[i] = NAN;
    distance[i] = NAN;
    return;
  }
  const uint64_t k0 = T / S;
  uint64_t bk = 0, bnum = 0;
  for (uint64_t kk = k0 > 1 ? k0 - 1 : 1; kk <= k0 + 2; ++kk) {
    const uint64_t a = S * kk;  // <= T + 2 S < 2^52
    const uint64_t num = a > T ? a - T : T - a;
    if (bk == 0 || (u128)num * bk < (u128)bnum * kk) {
      bk = kk;
      bnum = num;
    }
  }
  segments[i] = (uint32_t)bk;
  aligned[i] = (double)T / (double)bk;      // both exact in FP64
  distance[i] = (double)bnum / (double)T;   // bnum < 2^52: exact
}

// One wave per experiment, four per workgroup: lanes over the array sizes
// (a = lane + 64 t), strides in turn; the scores meet in LDS for lane 0.
__global__ __launch_bounds__(256) void line_kernel(const ks_desc* __restrict__ desc, uint32_t num_exp,
                                                   const ks_row_stats* __restrict__ stats, uint64_t stats_rows,
                                                   uint32_t J, const uint32_t* __restrict__ strides,
                                                   ks_line* __restrict__ out) {
  __shared__ uint64_t score[4][kLineMaxJ];
  const uint32_t lane = ks::lane_id(), w = ks::wave_id();
  const uint32_t e = blockIdx.x * 4u + w;
  if (e >= num_exp) return;
  const ks_desc d = desc[e];
  const uint32_t K = d.K, A = K / J;
  const bool bad = A < 1 || A > kLineMaxA || A * J != K || d.aux_offset > stats_rows ||
                   (uint64_t)K > stats_rows - d.aux_offset;
  if (bad) {
    if (lane == 0) out[e] = ks_line{0u, 0u, KS_LINE_INVALID, 0u, 0.0};
    return;
  }
  const ks_row_stats* x = stats + d.aux_offset;
  constexpr int T = kLineMaxA / ks::kWave;
  uint32_t P[T], M[T];
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const uint32_t a = lane + ks::kWave * (uint32_t)t;
    P[t] = a < A ? x[a].p50 : 0u;
    M[t] = a < A ? x[(uint64_t)(J - 1) * A + a].p50 : 0u;
  }
  for (uint32_t j = 0; j < J; ++j) {
    uint64_t acc = 0;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const uint32_t a = lane + ks::kWave * (uint32_t)t;
      if (a < A) {
        const uint32_t v = x[(uint64_t)j * A + a].p50;
        const uint64_t dp = v > P[t] ? v - P[t] : P[t] - v;
        const uint64_t dm = v > M[t] ? v - M[t] : M[t] - v;
        const uint64_t q = dp + dm ? (dp << 32) / (dp + dm) : 0ull;
        acc += (uint64_t)(a + 1) * q;  // < 2^8 * 2^32 per term, < 2^48 summed
      }
    }
    uint32_t unused = 0;
    ks::wave_total_32_64(unused, acc);
    if (lane == 0) score[w][j] = acc;
  }
  if (lane != 0) return;
  const uint64_t W = (uint64_t)A * (A + 1) / 2;
  const uint64_t half = W << 31;
  uint32_t jstar = J;
  for (uint32_t j = 1; j < J; ++j)
    if (score[w][j] > half) {
      jstar = j;
      break;
    }
  // adapted score: the running maximum from jstar on; increases between
  // consecutive power-of-two strides
  uint64_t run = 0, prev = 0;
  int64_t best = 0;
  uint32_t best_line = 0, ncand = 0, prev_stride = 0;
  for (uint32_t j = 0; j < J; ++j) {
    uint64_t sc = score[w][j];
    if (j >= jstar) {
      run = max(run, sc);
      sc = run;
    }
    const uint32_t st = strides[j];
    if (st == 0 || (st & (st - 1)) != 0) continue;
    if (ncand > 0) {
      const int64_t inc = (int64_t)sc - (int64_t)prev;
      if (ncand == 1 || inc > best) {
        best = inc;
        best_line = prev_stride;
      }
    }
    prev = sc;
    prev_stride = st;
    ++ncand;
  }
  uint32_t flags = jstar < J ? 0u : KS_LINE_NO_MAX_LIKE;
  if (ncand < 2) {
    out[e] = ks_line{0u, jstar, flags | KS_LINE_INCONCLUSIVE, 0u, 0.0};
    return;
  }
  if (best <= 0) flags |= KS_LINE_NO_INCREASE;
  out[e] = ks_line{best_line, jstar, flags, 0u, (double)best / (double)(W << 32)};
}

}  // namespace

extern "C" int ks_check_batch(ks_ctx* ctx, const ks_desc* desc, uint32_t num_series, uint32_t max_K,
                              const ks_result* res, const ks_row_stats* stats, uint64_t stats_rows, uint32_t edge,
                              uint32_t k, ks_check* out, void* stream) {
  if (!ctx) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (max_K < 2 || max_K > KS_MAX_K) return KS_E_RANGE;
  if (edge < 1 || k < 1) return KS_E_INVALID;
  if (num_series == 0) return KS_OK;
  if (!desc || !res || !stats || !out) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipLaunchKernelGGL(check_kernel, dim3((num_series + 3) / 4), dim3(256), 0, (hipStream_t)stream, desc, num_series,
                     max_K, res, stats, stats_rows, edge, k, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "check launch");
}

extern "C" int ks_align_batch(const uint64_t* measured, const uint64_t* total, uint32_t n, uint32_t* segments,
                              double* aligned, double* distance, void* stream) {
  if (n == 0) return KS_OK;
  if (!measured || !total || !segments || !aligned || !distance) return KS_E_INVALID;
  hipLaunchKernelGGL(align_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, measured, total, n,
                     segments, aligned, distance);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "align launch");
}

extern "C" int ks_line_batch(ks_ctx* ctx, const ks_desc* desc, uint32_t num_exp, const ks_row_stats* stats,
                             uint64_t stats_rows, uint32_t J, const uint32_t* strides, ks_line* out, void* stream) {
  if (!ctx) return KS_E_INVALID;
  if (J < 2 || J > kLineMaxJ) return KS_E_RANGE;
  if (num_exp == 0) return KS_OK;
  if (!desc || !stats || !strides || !out) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipLaunchKernelGGL(line_kernel, dim3((num_exp + 3) / 4), dim3(256), 0, (hipStream_t)stream, desc, num_exp, stats,
                     stats_rows, J, strides, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "line launch");
}

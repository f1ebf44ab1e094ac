// Batching of uneven series: an on-device plan, then either an ordered grid or
// a persistent launch.
//
// plan_kernel (one workgroup) turns the descriptors into work items, ordered
// largest first (bucketed by item size: a longest-processing-time order). A
// series whose samples fit in about `chunk_bytes` is one item, scanned start
// to end by one workgroup with its moments in LDS; a larger series is cut
// into whole row ranges (at most kMaxChunks items) whose per-row moments go
// to the workspace.
//
//   ordered grid  (chunk_bytes = no split): scan_kernel maps blockIdx to the
//                 ordered items, so the largest series are dispatched first;
//   persistent    scan_persistent drains the ordered items through an atomic
//                 queue with a grid sized to the resident capacity; then
//                 finish_kernel completes the split series from the
//                 workspace (the kernel boundary publishes the moments, so no
//                 device-scope fence is needed inside either kernel).
#pragma once

#include "ks_scan.hpp"

namespace ks {

struct Item {
  uint32_t series;
  uint16_t chunk;
  uint16_t nchunks;
};

// Device workspace (owned by the context), passed by value.
struct Workspace {
  uint32_t* hdr;       // [0] queue head, [1] number of items
  Item* items;         // kMaxChunks * num_series
  uint64_t* mom_base;  // per series: first RowMom slot (split series only)
  uint32_t* done;      // per series: completed items
  uint32_t* smin;      // per series: minimum over completed items
  RowMom* mom;         // per-row moments of split series
};

constexpr uint32_t kMaxChunks = 64;
constexpr int kPlanNT = 1024;
constexpr int kBuckets = 48;
constexpr uint32_t kNoSplit = 0xffffffffu;  // chunk_bytes of the ordered grid: one item per series

// Rows per work item: whole rows, about chunk_bytes of samples, at most
// kMaxChunks items per series; the whole series when chunk_bytes is kNoSplit
// (the ordered grid dispatches exactly one workgroup per series, so a series
// of more than 4 GiB must not become several items there).
__device__ __forceinline__ uint32_t rows_per_item(uint32_t K, uint32_t N, uint32_t chunk_bytes) {
  if (chunk_bytes == kNoSplit) return K;
  uint64_t rpc = chunk_bytes / (4ull * N);
  if (rpc < 1) rpc = 1;
  const uint32_t minr = (K + kMaxChunks - 1) / kMaxChunks;
  if (rpc < minr) rpc = minr;
  return rpc >= K ? K : (uint32_t)rpc;
}

__device__ __forceinline__ void item_shape(const ks_desc& d, uint64_t num_samples, uint32_t max_K,
                                           uint32_t chunk_bytes, uint32_t& nc, uint32_t& bucket) {
  uint64_t bytes = 0;
  nc = 1;
  if (!check_desc(d, num_samples, max_K)) {
    const uint32_t rpc = rows_per_item(d.K, d.N, chunk_bytes);
    nc = (d.K + rpc - 1) / rpc;
    bytes = 4ull * rpc * d.N;
  }
  const int bl = bytes ? 64 - __clzll(bytes) : 0;  // larger items -> smaller bucket index
  bucket = (uint32_t)(kBuckets - 1 - (bl < kBuckets - 1 ? bl : kBuckets - 1));
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const uint32_t l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t t = (uint64_t)__shfl_up((unsigned long long)v, o);
    if (l >= (uint32_t)o) v += t;
  }
  return v;
}

static __global__ __launch_bounds__(kPlanNT) void plan_kernel(const ks_desc* __restrict__ desc, uint32_t S,
                                                       uint64_t num_samples, uint32_t max_K, uint32_t chunk_bytes,
                                                       Workspace ws) {
  __shared__ uint32_t hist[kBuckets];
  __shared__ uint32_t start[kBuckets];
  __shared__ uint64_t wsum[kPlanNT / kWave];
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = wave_id();
  for (uint32_t b = tid; b < (uint32_t)kBuckets; b += kPlanNT) hist[b] = 0;
  __syncthreads();
  const uint32_t per = (S + kPlanNT - 1) / kPlanNT;
  const uint32_t s0 = min(S, tid * per), s1 = min(S, s0 + per);
  uint64_t rows = 0;
  for (uint32_t s = s0; s < s1; ++s) {
    const ks_desc d = desc[s];
    uint32_t nc, b;
    item_shape(d, num_samples, max_K, chunk_bytes, nc, b);
    if (nc > 1) rows += d.K;
    atomicAdd(&hist[b], nc);
    ws.done[s] = 0;
    ws.smin[s] = 0xffffffffu;
  }
  const uint64_t incl = wave_incl_scan_u64(rows);
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint64_t base = incl - rows;
  for (uint32_t v = 0; v < w; ++v) base += wsum[v];
  if (tid == 0) {
    uint32_t run = 0;
    for (int b = 0; b < kBuckets; ++b) {
      start[b] = run;
      run += hist[b];
    }
    ws.hdr[0] = 0;
    ws.hdr[1] = run;
  }
  __syncthreads();
  for (uint32_t s = s0; s < s1; ++s) {
    const ks_desc d = desc[s];
    uint32_t nc, b;
    item_shape(d, num_samples, max_K, chunk_bytes, nc, b);
    const uint32_t pos = atomicAdd(&start[b], nc);
    for (uint32_t c = 0; c < nc; ++c) ws.items[pos + c] = Item{s, (uint16_t)c, (uint16_t)nc};
    ws.mom_base[s] = base;
    if (nc > 1) base += d.K;
  }
}

template <int KMAX, int NT, int RB, int GM = 0>
__global__ __launch_bounds__(NT) void scan_persistent(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                      const ks_desc* __restrict__ desc, uint32_t num_series,
                                                      ks_params prm, uint32_t max_K, ks_result* __restrict__ out,
                                                      uint32_t* __restrict__ allU, uint64_t allU_len,
                                                      uint32_t chunk_bytes, Workspace ws) {
  using S = ScanShape<KMAX, NT, RB>;
  __shared__ ScanSmem<KMAX, NT, RB> sm;
  __shared__ uint32_t s_item;
  // the plan writes at most kMaxChunks items per series
  const uint32_t cap = num_series <= 0xffffffffu / kMaxChunks ? num_series * kMaxChunks : 0xffffffffu;
  const uint32_t total = min(ws.hdr[1], cap);
  const uint32_t lane = lane_id(), w = wave_id();
  for (;;) {
    // The barrier at the top of every iteration keeps the queue fetch below
    // from sitting next to any thread-0-only branch at the end of the
    // previous iteration: without it the compiler may route threads != 0
    // around the fetch into an inner loop that never sees a new item.
    __syncthreads();
    if (threadIdx.x == 0) s_item = atomicAdd(&ws.hdr[0], 1u);
    __syncthreads();
    const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
    if (it >= total) break;
    const Item item = ws.items[it];
    const uint32_t s = __builtin_amdgcn_readfirstlane(item.series);
    if (s >= num_series) continue;
    const ks_desc d = desc[s];
    if (item.nchunks <= 1 || check_desc(d, num_samples, max_K)) {
      scan_one<KMAX, NT, RB, GM>(sm, samples, num_samples, d, prm, max_K, out + s, allU, allU_len);
      continue;
    }
    // one row range of a split series: moments to the workspace
    const uint32_t K = d.K, N = d.N;
    const uint32_t rpc = rows_per_item(K, N, chunk_bytes);
    const uint32_t r0 = (uint32_t)item.chunk * rpc, r1 = min(K, r0 + rpc);
    RowMom* mom = ws.mom + ws.mom_base[s];
    const uint32_t mn = stream_rows(samples, d.offset, N, r0 + w, r1, S::W, lane,
                                    [&](uint32_t i, uint64_t s1, uint64_t s2, uint32_t s2h, uint32_t) {
                                      if (lane == 0) {
                                        mom[i].s1 = s1;
                                        mom[i].s2lo = s2;
                                        mom[i].s2hi = s2h;
                                      }
                                    });
    const uint32_t g = block_min_u32<NT>(mn, sm.red);
    if (threadIdx.x == 0) atomicMin(&ws.smin[s], g);
  }
}

// Completes the series that the plan split (one workgroup per series; the
// others return at once): gathers their moments and runs keys, sort, walk,
// choice and p-value.
template <int KMAX, int NT, int RB, int GM = 0>
__global__ __launch_bounds__(NT) void finish_kernel(uint64_t num_samples, const ks_desc* __restrict__ desc,
                                                    uint32_t num_series, ks_params prm, uint32_t max_K,
                                                    ks_result* __restrict__ out, uint32_t* __restrict__ allU,
                                                    uint64_t allU_len, uint32_t chunk_bytes, Workspace ws) {
  __shared__ ScanSmem<KMAX, NT, RB> sm;
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  uint32_t nc, b;
  item_shape(d, num_samples, max_K, chunk_bytes, nc, b);
  if (nc <= 1) return;
  const uint32_t K = d.K;
  const RowMom* mom = ws.mom + ws.mom_base[s];
  for (uint32_t i = threadIdx.x; i < K; i += NT) {
    sm.u.mom.s1[i] = mom[i].s1;
    sm.u.mom.s2lo[i] = mom[i].s2lo;
    sm.u.mom.s2hi[i] = mom[i].s2hi;
  }
  const uint32_t gmin = ws.smin[s];
  __syncthreads();
  const bool fits = allU && d.aux_offset <= allU_len && K <= allU_len - d.aux_offset;
  finish_series<KMAX, NT, RB, GM>(sm, K, d.N, gmin, prm, out + s, fits ? allU + d.aux_offset : nullptr);
}

}  // namespace ks

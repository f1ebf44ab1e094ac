// Binary segmentation over a batch: every level boundary of each series.
// Depth 0 scans the whole series like ks_scan_batch and also keeps every
// row's moments and minimum (24 B per row). A window [a, b) of a later depth
// is a series of its own, but its eq. 2 keys need only its rows' sum r and
// sum r^2 and the window's minimum (the least row minimum), so depths >= 1
// read that workspace and never the samples. After each depth a split kernel
// records the significant splits and opens both sides of each as windows of
// the next depth; a final kernel sorts each series' boundaries by position.
// Window and split kernels run on fixed grids that stride over the depth's
// window count in device memory, so the host enqueues several depths between
// read-backs of those counts.
#include <hip/hip_runtime.h>

#include <new>

#include "ks.h"
#include "ks_ctx.hpp"
#include "ks_scan.hpp"
#include "ks_wave.hpp"

using namespace ks_host;

namespace ks_host {

void free_seg(SegBuffers& b) {
  void* dev[] = {b.win[0], b.win[1], b.wser[0], b.wser[1], b.wstart[0], b.wstart[1], b.res, b.ctr, b.rows};
  for (void* p : dev) (void)hipFree(p);
  if (b.host_ctr) (void)hipHostFree(b.host_ctr);
  b = SegBuffers{};
}

}  // namespace ks_host

namespace {

constexpr uint32_t kSegNT = 256;
constexpr uint32_t kSegGrid = 2048;      // workgroups of a window-scan launch (grid-stride over the windows)
constexpr uint32_t kSegSplitGrid = 256;  // workgroups of a split launch
constexpr uint32_t kSegDepths = KS_MAX_K + 1;  // counter pairs: a window of a later depth is a part of one before it

// Depth 0: the full scan of series blockIdx.x (as scan_kernel, in workgroups
// of kSegRootNT threads: the streaming depth is HBM-bound like the plain
// scan), also storing each row's moments and minimum at rows[s * row_stride + i].
// The rows' minima wait in the key buffer (free until the keys are made) and
// the records are written once the series is streamed, consecutive threads
// taking consecutive rows, rather than one 24-byte store per row as it ends.
constexpr int kSegRootNT = 512;

template <int KMAX>
__global__ __launch_bounds__(kSegRootNT) void seg_root_kernel(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                       const ks_desc* __restrict__ desc, uint32_t num_series,
                                                       ks_params prm, uint32_t max_K, ks_result* __restrict__ out,
                                                       ks::RowMom* __restrict__ rows, uint32_t row_stride) {
  using S = ks::ScanShape<KMAX, kSegRootNT, kRB>;
  __shared__ ks::ScanSmem<KMAX, kSegRootNT, kRB> sm;
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const uint32_t bad = ks::check_desc(d, num_samples, max_K);
  if (bad) {
    if (threadIdx.x == 0) ks::write_result(out + s, 0, 0, 0, 0, 0.0, 0.0, 1.0, bad);
    return;
  }
  const uint32_t lane = ks::lane_id(), w = ks::wave_id();
  ks::RowMom* rm = rows + (uint64_t)s * row_stride;
  const uint32_t mn = ks::stream_rows<true>(samples, d.offset, d.N, w, d.K, S::W, lane,
                                            [&](uint32_t i, uint64_t s1, uint64_t s2, uint32_t s2h, uint32_t rmin) {
                                              if (lane == 0) {
                                                sm.u.mom.s1[i] = s1;
                                                sm.u.mom.s2lo[i] = s2;
                                                sm.u.mom.s2hi[i] = s2h;
                                                sm.key[0][i] = rmin;
                                              }
                                            });
  const uint32_t gmin = ks::block_min_u32<kSegRootNT>(mn, sm.red);  // its barriers publish the rows
  for (uint32_t i = threadIdx.x; i < d.K; i += kSegRootNT)
    rm[i] = ks::RowMom{sm.u.mom.s1[i], sm.u.mom.s2lo[i], sm.u.mom.s2hi[i], sm.key[0][i]};
  __syncthreads();  // the minima are read before the keys overwrite them
  ks::finish_series(sm, d.K, d.N, gmin, prm, out + s, nullptr);
}

// Depth >= 1: windows t = blockIdx.x, + gridDim.x, ... below *count (series
// wser[t], rows wstart[t] .. + win[t].K) from the stored row moments; a
// window's eq. 2 minimum is the least of its rows' minima.
template <int KMAX>
__global__ __launch_bounds__(kNT) void seg_window_kernel(const ks_desc* __restrict__ win,
                                                         const uint32_t* __restrict__ count,
                                                         const uint32_t* __restrict__ wser,
                                                         const uint32_t* __restrict__ wstart, ks_params prm,
                                                         const ks::RowMom* __restrict__ rows, uint32_t row_stride,
                                                         ks_result* __restrict__ out) {
  __shared__ ks::ScanSmem<KMAX, kNT, kRB> sm;
  const uint32_t n = *count;
  for (uint32_t t = blockIdx.x; t < n; t += gridDim.x) {
    __syncthreads();  // the previous window's reads of sm are done
    const ks_desc d = win[t];
    const uint32_t K = d.K;
    if (K < 2 || K > (uint32_t)KMAX) {  // never opened by the split kernel
      if (threadIdx.x == 0) ks::write_result(out + t, 0, 0, 0, 0, 0.0, 0.0, 1.0, KS_BAD_SHAPE);
      continue;
    }
    const ks::RowMom* rm = rows + (uint64_t)wser[t] * row_stride + wstart[t];
    uint32_t mn = 0xffffffffu;
    for (uint32_t i = threadIdx.x; i < K; i += kNT) {
      const ks::RowMom r = rm[i];
      sm.u.mom.s1[i] = r.s1;
      sm.u.mom.s2lo[i] = r.s2lo;
      sm.u.mom.s2hi[i] = r.s2hi;
      mn = min(mn, r.pad);
    }
    const uint32_t gmin = ks::block_min_u32<kNT>(mn, sm.red);  // its barriers also publish the moments
    ks::finish_series(sm, K, d.N, gmin, prm, out + t, nullptr);
  }
}

template <template <int> class KERNEL, typename... Args>
void launch_kc(int kc, uint32_t grid, hipStream_t st, Args... args) {
  switch (kc) {
    case 0: hipLaunchKernelGGL(KERNEL<64>::f, dim3(grid), dim3(KERNEL<64>::nt), 0, st, args...); break;
    case 1: hipLaunchKernelGGL(KERNEL<128>::f, dim3(grid), dim3(KERNEL<128>::nt), 0, st, args...); break;
    case 2: hipLaunchKernelGGL(KERNEL<256>::f, dim3(grid), dim3(KERNEL<256>::nt), 0, st, args...); break;
    case 3: hipLaunchKernelGGL(KERNEL<512>::f, dim3(grid), dim3(KERNEL<512>::nt), 0, st, args...); break;
    case 4: hipLaunchKernelGGL(KERNEL<1024>::f, dim3(grid), dim3(KERNEL<1024>::nt), 0, st, args...); break;
    default: hipLaunchKernelGGL(KERNEL<2048>::f, dim3(grid), dim3(KERNEL<2048>::nt), 0, st, args...);
  }
}
template <int KMAX>
struct RootK {
  static constexpr auto f = seg_root_kernel<KMAX>;
  static constexpr int nt = kSegRootNT;
};
template <int KMAX>
struct WindowK {
  static constexpr auto f = seg_window_kernel<KMAX>;
  static constexpr int nt = kNT;
};

// One thread per open window of depth `depth` (n of them, or *count when
// count is given), grid-stride. Window t is series wser[t] (t itself at
// depth 0) starting at row wstart[t] (0 at depth 0). ctr: the next depth's
// window count and largest K.
__global__ __launch_bounds__(kSegNT) void seg_split_kernel(
    const ks_desc* __restrict__ win, const ks_result* __restrict__ res, uint32_t n, const uint32_t* __restrict__ count,
    const uint32_t* __restrict__ wser, const uint32_t* __restrict__ wstart, uint32_t depth, int open_next,
    ks_desc* __restrict__ next, uint32_t* __restrict__ nser, uint32_t* __restrict__ nstart, uint32_t* __restrict__ ctr,
    uint64_t cap, ks_result* __restrict__ cps, uint32_t* __restrict__ counts, uint32_t max_cp) {
  if (count) n = *count;
  for (uint32_t t = blockIdx.x * kSegNT + threadIdx.x; t < n; t += gridDim.x * kSegNT) {
  const ks_result r = res[t];
  const uint32_t s = wser ? wser[t] : t;
  const uint32_t a = wstart ? wstart[t] : 0u;
  if (r.flags & (KS_BAD_SHAPE | KS_OUT_OF_RANGE)) {
    // only a caller's descriptor can be malformed: every later window lies inside a valid series
    if (depth == 0) counts[s] = KS_SEGMENT_BAD;
    continue;
  }
  if (!(r.flags & KS_SIGNIFICANT)) continue;
  const ks_desc d = win[t];
  const uint32_t slot = atomicAdd(&counts[s], 1u);
  if (slot < max_cp) {
    ks_result o = r;
    o.cp = a + r.cp;
    o.pad = depth;
    cps[(uint64_t)s * max_cp + slot] = o;
  }
  if (!open_next) continue;
  const uint32_t kl = r.cp, kr = d.K - r.cp;
  if (kl >= 2) {
    const uint32_t i = atomicAdd(&ctr[0], 1u);
    if (i < cap) {
      next[i] = ks_desc{d.offset, kl, d.N, 0};
      nser[i] = s;
      nstart[i] = a;
      atomicMax(&ctr[1], kl);
    }
  }
  if (kr >= 2) {
    const uint32_t i = atomicAdd(&ctr[0], 1u);
    if (i < cap) {
      next[i] = ks_desc{d.offset + (uint64_t)r.cp * d.N, kr, d.N, 0};
      nser[i] = s;
      nstart[i] = a + r.cp;
      atomicMax(&ctr[1], kr);
    }
  }
  }
}

// Sort each series' stored boundaries by cp (insertion sort; one thread per
// series, positions are distinct).
__global__ __launch_bounds__(kSegNT) void seg_sort_kernel(ks_result* __restrict__ cps,
                                                          const uint32_t* __restrict__ counts, uint32_t num_series,
                                                          uint32_t max_cp) {
  const uint32_t s = blockIdx.x * kSegNT + threadIdx.x;
  if (s >= num_series) return;
  const uint32_t c = counts[s];
  if (c == KS_SEGMENT_BAD) return;
  const uint32_t k = c < max_cp ? c : max_cp;
  ks_result* v = cps + (uint64_t)s * max_cp;
  for (uint32_t i = 1; i < k; ++i) {
    const ks_result x = v[i];
    uint32_t j = i;
    while (j > 0 && v[j - 1].cp > x.cp) {
      v[j] = v[j - 1];
      --j;
    }
    v[j] = x;
  }
}

template <typename T>
bool alloc(T*& p, uint64_t n) {
  return hipMalloc(&p, sizeof(T) * (n ? n : 1)) == hipSuccess;
}

int ensure_seg(ks_ctx* c, uint64_t cap, uint64_t rows) {
  SegBuffers& b = c->seg;
  if (cap <= b.cap && rows <= b.cap_rows) return KS_OK;
  if (cap < b.cap) cap = b.cap;
  if (rows < b.cap_rows) rows = b.cap_rows;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  free_seg(b);
  bool ok = alloc(b.win[0], cap) && alloc(b.win[1], cap) && alloc(b.wser[0], cap) && alloc(b.wser[1], cap) &&
            alloc(b.wstart[0], cap) && alloc(b.wstart[1], cap) && alloc(b.res, cap) &&
            alloc(b.ctr, 2 * kSegDepths) && alloc(b.rows, rows) &&
            hipHostMalloc(reinterpret_cast<void**>(&b.host_ctr), 2 * kSegDepths * sizeof(uint32_t),
                          hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    free_seg(b);
    (void)hipGetLastError();
    return KS_E_NOMEM;
  }
  b.cap = cap;
  b.cap_rows = rows;
  return KS_OK;
}

}  // namespace

extern "C" int ks_segment_batch(ks_ctx* ctx, const uint32_t* samples, uint64_t num_samples, const ks_desc* desc,
                                uint32_t num_series, const ks_params* params, uint32_t max_levels, uint32_t max_cp,
                                ks_result* cps, uint32_t* counts, void* stream) {
  if (!ctx || !params) return KS_E_INVALID;
  if (int rc = check_params(params)) return rc;
  if (num_series == 0) return KS_OK;
  if (!samples || !desc || !cps || !counts || max_cp == 0) return KS_E_INVALID;
  const uint32_t max_K = params->max_K ? params->max_K : KS_MAX_K;
  if (max_K < 2 || max_K > KS_MAX_K) return KS_E_RANGE;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  // the windows of one depth are disjoint row ranges of >= 2 rows of their series
  const uint64_t cap = (uint64_t)num_series * (max_K / 2 > 1 ? max_K / 2 : 1);
  if (int rc = ensure_seg(ctx, cap, (uint64_t)num_series * max_K)) return rc;
  SegBuffers& b = ctx->seg;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemsetAsync(counts, 0, sizeof(uint32_t) * num_series, st);
  if (e != hipSuccess) return hip_fail(e, "counts reset");
  if ((e = hipMemsetAsync(b.ctr, 0, 2 * sizeof(uint32_t) * kSegDepths, st)) != hipSuccess)
    return hip_fail(e, "window counters");
  // a window of depth d >= 1 has at most max_K - d rows, so depth max_K - 1 opens none
  const uint32_t limit = max_levels == 0 || max_levels > max_K - 1 ? max_K - 1 : max_levels;
  const uint32_t wgrid = (uint32_t)(b.cap < kSegGrid ? b.cap : kSegGrid);
  const uint32_t sgrid = (uint32_t)((b.cap + kSegNT - 1) / kSegNT < kSegSplitGrid ? (b.cap + kSegNT - 1) / kSegNT
                                                                                     : kSegSplitGrid);
  // depth 0: every series
  launch_kc<RootK>(k_class(max_K), num_series, st, samples, num_samples, desc, num_series, *params, max_K, b.res,
                   b.rows, max_K);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "root scan launch");
  hipLaunchKernelGGL(seg_split_kernel, dim3((num_series + kSegNT - 1) / kSegNT), dim3(kSegNT), 0, st, desc, b.res,
                     num_series, (const uint32_t*)nullptr, (const uint32_t*)nullptr, (const uint32_t*)nullptr, 0u,
                     (int)(limit > 1), b.win[0], b.wser[0], b.wstart[0], b.ctr + 2, b.cap, cps, counts, max_cp);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "split launch");
  // later depths in chunks of 4, 8, 16, ... between read-backs of their window counts; a
  // depth whose count is 0 costs two near-empty launches
  uint32_t roundK = max_K;
  uint32_t depth = 1, chunk = 4;
  while (depth < limit) {
    const uint32_t end = depth + chunk < limit ? depth + chunk : limit;
    for (uint32_t d = depth; d < end; ++d) {
      const int src = (d - 1) & 1, dst = d & 1;
      launch_kc<WindowK>(k_class(roundK), wgrid, st, b.win[src], (const uint32_t*)(b.ctr + 2 * d), b.wser[src],
                         b.wstart[src], *params, (const ks::RowMom*)b.rows, max_K, b.res);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "window scan launch");
      hipLaunchKernelGGL(seg_split_kernel, dim3(sgrid), dim3(kSegNT), 0, st, b.win[src], b.res, 0u,
                         (const uint32_t*)(b.ctr + 2 * d), b.wser[src], b.wstart[src], d, (int)(d + 1 < limit),
                         b.win[dst], b.wser[dst], b.wstart[dst], b.ctr + 2 * (d + 1), b.cap, cps, counts, max_cp);
      if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "split launch");
    }
    // counts of depths depth + 1 .. end
    if ((e = hipMemcpyAsync(b.host_ctr, b.ctr + 2 * (depth + 1), 2 * sizeof(uint32_t) * (end - depth),
                            hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "window count");
    bool open = false;
    for (uint32_t d = 0; d < end - depth; ++d) {
      if (b.host_ctr[2 * d] > b.cap) return KS_E_STATE;  // cannot happen: windows of a depth are disjoint
      open = b.host_ctr[2 * d] > 0;
      if (open && b.host_ctr[2 * d + 1] >= 2) roundK = b.host_ctr[2 * d + 1];
    }
    if (!open) break;
    depth = end;
    chunk *= 2;
  }
  hipLaunchKernelGGL(seg_sort_kernel, dim3((num_series + kSegNT - 1) / kSegNT), dim3(kSegNT), 0, st, cps, counts,
                     num_series, max_cp);
  e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "sort launch");
}

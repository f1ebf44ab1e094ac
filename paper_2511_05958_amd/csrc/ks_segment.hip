// Binary segmentation over a batch: every level boundary of each series.
// Depth by depth, all open windows of the batch are scanned by one
// ks_scan_batch (each window a series of its own, with its own eq. 2
// minimum); a split kernel records the significant splits and opens the two
// sides of each as windows of the next depth; a final kernel sorts each
// series' boundaries by position.
#include <hip/hip_runtime.h>

#include <new>

#include "ks.h"
#include "ks_ctx.hpp"
#include "ks_wave.hpp"

using namespace ks_host;

namespace ks_host {

void free_seg(SegBuffers& b) {
  void* dev[] = {b.win[0], b.win[1], b.wser[0], b.wser[1], b.wstart[0], b.wstart[1], b.res, b.ctr};
  for (void* p : dev) (void)hipFree(p);
  if (b.host_ctr) (void)hipHostFree(b.host_ctr);
  b = SegBuffers{};
}

}  // namespace ks_host

namespace {

constexpr uint32_t kSegNT = 256;

// One thread per open window of depth `depth`. Window t is series wser[t]
// (t itself at depth 0) starting at row wstart[t] (0 at depth 0).
__global__ __launch_bounds__(kSegNT) void seg_split_kernel(
    const ks_desc* __restrict__ win, const ks_result* __restrict__ res, uint32_t n,
    const uint32_t* __restrict__ wser, const uint32_t* __restrict__ wstart, uint32_t depth, int open_next,
    ks_desc* __restrict__ next, uint32_t* __restrict__ nser, uint32_t* __restrict__ nstart, uint32_t* __restrict__ ctr,
    uint64_t cap, ks_result* __restrict__ cps, uint32_t* __restrict__ counts, uint32_t max_cp) {
  const uint32_t t = blockIdx.x * kSegNT + threadIdx.x;
  if (t >= n) return;
  const ks_result r = res[t];
  const uint32_t s = wser ? wser[t] : t;
  const uint32_t a = wstart ? wstart[t] : 0u;
  if (r.flags & (KS_BAD_SHAPE | KS_OUT_OF_RANGE)) {
    // only a caller's descriptor can be malformed: every later window lies inside a valid series
    if (depth == 0) counts[s] = KS_SEGMENT_BAD;
    return;
  }
  if (!(r.flags & KS_SIGNIFICANT)) return;
  const ks_desc d = win[t];
  const uint32_t slot = atomicAdd(&counts[s], 1u);
  if (slot < max_cp) {
    ks_result o = r;
    o.cp = a + r.cp;
    o.pad = depth;
    cps[(uint64_t)s * max_cp + slot] = o;
  }
  if (!open_next) return;
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

int ensure_seg(ks_ctx* c, uint64_t cap) {
  SegBuffers& b = c->seg;
  if (cap <= b.cap) return KS_OK;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  free_seg(b);
  bool ok = alloc(b.win[0], cap) && alloc(b.win[1], cap) && alloc(b.wser[0], cap) && alloc(b.wser[1], cap) &&
            alloc(b.wstart[0], cap) && alloc(b.wstart[1], cap) && alloc(b.res, cap) && alloc(b.ctr, 2) &&
            hipHostMalloc(reinterpret_cast<void**>(&b.host_ctr), 2 * sizeof(uint32_t), hipHostMallocDefault) ==
                hipSuccess;
  if (!ok) {
    free_seg(b);
    (void)hipGetLastError();
    return KS_E_NOMEM;
  }
  b.cap = cap;
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
  if (int rc = ensure_seg(ctx, cap)) return rc;
  SegBuffers& b = ctx->seg;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemsetAsync(counts, 0, sizeof(uint32_t) * num_series, st);
  if (e != hipSuccess) return hip_fail(e, "counts reset");
  const ks_desc* cur = desc;
  const uint32_t* cser = nullptr;
  const uint32_t* cstart = nullptr;
  uint64_t n = num_series;
  uint32_t roundK = max_K;
  int dst = 0;
  for (uint32_t depth = 0; n > 0 && (max_levels == 0 || depth < max_levels); ++depth) {
    ks_params p = *params;
    p.max_K = roundK;
    if (int rc = ks_scan_batch(ctx, samples, num_samples, cur, (uint32_t)n, &p, b.res, nullptr, 0, stream)) return rc;
    const int open_next = max_levels == 0 || depth + 1 < max_levels;
    if ((e = hipMemsetAsync(b.ctr, 0, 2 * sizeof(uint32_t), st)) != hipSuccess) return hip_fail(e, "window counter");
    hipLaunchKernelGGL(seg_split_kernel, dim3((uint32_t)((n + kSegNT - 1) / kSegNT)), dim3(kSegNT), 0, st, cur, b.res,
                       (uint32_t)n, cser, cstart, depth, open_next, b.win[dst], b.wser[dst], b.wstart[dst], b.ctr, b.cap,
                       cps, counts, max_cp);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "split launch");
    if (!open_next) break;
    if ((e = hipMemcpyAsync(b.host_ctr, b.ctr, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "window count");
    if (b.host_ctr[0] > b.cap) return KS_E_STATE;  // cannot happen: windows of a depth are disjoint
    n = b.host_ctr[0];
    roundK = b.host_ctr[1] >= 2 ? b.host_ctr[1] : 2;
    cur = b.win[dst];
    cser = b.wser[dst];
    cstart = b.wstart[dst];
    dst ^= 1;
  }
  hipLaunchKernelGGL(seg_sort_kernel, dim3((num_series + kSegNT - 1) / kSegNT), dim3(kSegNT), 0, st, cps, counts,
                     num_series, max_cp);
  e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "sort launch");
}

// Learned-proposal stage 1: one read of every sample gives, per row,
//   - the moments (sum r, sum r^2) that the exact refine turns into eq. 2 keys,
//   - the nine deciles x_(floor(k (N-1) / 10)), k = 1..9, from an LDS radix
//     sort of the row's uint32 cycle counts (keys r - row minimum, as many
//     RB-bit passes as the row's range needs),
// and per series the minimum m, then features f = (double)(x - m) / max(m, 1)
// rounded to float (project-defined inputs of the network).
#pragma once

#include "ks_cnn.hpp"
#include "ks_scan.hpp"

namespace ks {

// Per-row moments of the learned path (the refine's input), per-series min.
struct LearnWs {
  uint64_t* s1;     // [num_series * SR] (row slot of series s: s * SR + 2 + i)
  uint64_t* s2lo;
  uint32_t* s2hi;
  uint32_t* smin;   // [num_series]
  uint32_t* K;      // [num_series]: K when the series was valid, 0 otherwise
};

template <int NMAX, int NT, int RB>
struct RowSortShape {
  static constexpr int W = NT / kWave;
  static constexpr int E = (NMAX + NT - 1) / NT;  // samples per thread
  static constexpr int D = 1 << RB;
  static constexpr int H = D * E * W;
};

template <int NMAX, int NT, int RB>
struct FeatSmem {
  using S = RowSortShape<NMAX, NT, RB>;
  uint32_t key[2][NMAX];
  uint16_t hist[S::H];
  uint32_t red[S::W * 8];
  uint32_t dec[9];
};

// Block-wide stable LSD radix sort of n <= NMAX uint32 keys held as E per
// thread (element e of thread t is item e*NT + t). The sorted keys end in
// sm.key[result].
template <int NMAX, int NT, int RB>
__device__ int block_sort_u32(FeatSmem<NMAX, NT, RB>& sm, uint32_t (&v)[RowSortShape<NMAX, NT, RB>::E], uint32_t n,
                              int bits) {
  using S = RowSortShape<NMAX, NT, RB>;
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  constexpr int C = (S::H + NT - 1) / NT;
  const int passes = (bits + RB - 1) / RB;
  int cur = 0;
#pragma unroll
  for (int e = 0; e < S::E; ++e) {
    const uint32_t item = e * NT + tid;
    if (item < n) sm.key[0][item] = v[e];
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RB;
    for (int h = tid; h < S::H; h += NT) sm.hist[h] = 0;
    __syncthreads();
    uint32_t dg[S::E], rk[S::E];
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint32_t item = e * NT + tid;
      const bool valid = item < n;
      const uint32_t d = valid ? (sm.key[cur][item] >> shift) & (S::D - 1) : 0u;
      uint64_t peers = ballot(valid);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
      }
      dg[e] = d;
      rk[e] = mbcnt(peers);
      if (valid && rk[e] == 0) sm.hist[(d * S::E + e) * S::W + w] = (uint16_t)__popcll(peers);
    }
    __syncthreads();
    uint32_t local = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int h = tid * C + c;
      if (h < S::H) local += sm.hist[h];
    }
    const uint32_t incl = wave_incl_scan(local);
    if (lane == kWave - 1) sm.red[w] = incl;
    __syncthreads();
    uint32_t run = incl - local;
    for (uint32_t u = 0; u < w; ++u) run += sm.red[u];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int h = tid * C + c;
      if (h < S::H) {
        const uint32_t x = sm.hist[h];
        sm.hist[h] = (uint16_t)run;
        run += x;
      }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint32_t item = e * NT + tid;
      if (item < n) sm.key[cur ^ 1][sm.hist[(dg[e] * S::E + e) * S::W + w] + rk[e]] = sm.key[cur][item];
    }
    __syncthreads();
    cur ^= 1;
  }
  return cur;
}

// Features of one series per workgroup. Writes: the caller's FP32 features
// (nullable, rows at aux_offset), the network input rows (bf16, 16 channels,
// 9 used) at row slot s * SR + 2 + i, and the refine workspace.
template <int NMAX, int NT, int RB>
__global__ __launch_bounds__(NT) void features_kernel(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                      const ks_desc* __restrict__ desc, uint32_t num_series,
                                                      uint32_t max_K, float* __restrict__ feat_out,
                                                      uint64_t feat_rows, uint16_t* __restrict__ x0,
                                                      uint32_t SR, LearnWs lw, float* __restrict__ feat_ws) {
  using S = RowSortShape<NMAX, NT, RB>;
  __shared__ FeatSmem<NMAX, NT, RB> sm;
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
  if (check_desc(d, num_samples, max_K) || d.N > (uint32_t)NMAX) {
    for (uint32_t q = tid; q < SR * 16; q += NT) x0[(uint64_t)s * SR * 16 + q] = 0;
    if (tid == 0) lw.K[s] = 0;
    return;
  }
  const uint32_t K = d.K, N = d.N;
  const uint64_t slot = (uint64_t)s * SR + 2;
  uint32_t gmin = 0xffffffffu;
  for (uint32_t i = 0; i < K; ++i) {
    const uint32_t* row = samples + d.offset + (uint64_t)i * N;
    uint32_t v[S::E];
    uint32_t mn = 0xffffffffu, mx = 0;
    uint64_t s1 = 0, s2 = 0;
    uint32_t s2h = 0;
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint32_t j = e * NT + tid;
      v[e] = j < N ? __builtin_nontemporal_load(row + j) : 0u;
    }
#pragma unroll
    for (int e = 0; e < S::E; ++e) {
      const uint32_t j = e * NT + tid;
      if (j < N) {
        acc_sample(v[e], mn, s1, s2, s2h);
        mx = max(mx, v[e]);
      }
    }
    wave_total_64_96(s1, s2, s2h);
    mn = wave_min_u32(mn);
    mx = wave_max_u32(mx);
    if (lane == 0) {
      sm.red[w * 8 + 0] = mn;
      sm.red[w * 8 + 1] = mx;
      sm.red[w * 8 + 2] = (uint32_t)s1;
      sm.red[w * 8 + 3] = (uint32_t)(s1 >> 32);
      sm.red[w * 8 + 4] = (uint32_t)s2;
      sm.red[w * 8 + 5] = (uint32_t)(s2 >> 32);
      sm.red[w * 8 + 6] = s2h;
    }
    __syncthreads();
    uint32_t rmin = sm.red[0], rmax = sm.red[1];
    uint64_t t1 = 0, t2 = 0;
    uint32_t t2h = 0;
    for (int u = 0; u < S::W; ++u) {
      rmin = min(rmin, sm.red[u * 8 + 0]);
      rmax = max(rmax, sm.red[u * 8 + 1]);
      t1 += ((uint64_t)sm.red[u * 8 + 3] << 32) | sm.red[u * 8 + 2];
      const uint64_t a = ((uint64_t)sm.red[u * 8 + 5] << 32) | sm.red[u * 8 + 4];
      const uint64_t b = t2 + a;
      t2h += sm.red[u * 8 + 6] + (uint32_t)(b < t2);
      t2 = b;
    }
    __syncthreads();
    if (tid == 0) {
      lw.s1[slot + i] = t1;
      lw.s2lo[slot + i] = t2;
      lw.s2hi[slot + i] = t2h;
    }
    gmin = min(gmin, rmin);
    // sort keys r - rmin; only the range's bit length takes passes
    const uint32_t range = rmax - rmin;
    const int bits = range ? 32 - __clz(range) : 0;
#pragma unroll
    for (int e = 0; e < S::E; ++e) v[e] -= rmin;
    const int cur = block_sort_u32(sm, v, N, bits);
    if (tid < 9) {
      const uint32_t k = tid + 1;
      const uint32_t pos = (uint32_t)(((uint64_t)k * (N - 1)) / 10);
      // feature numerators x - m need the series minimum: keep x itself
      feat_ws[(slot + i) * 9 + tid] = __uint_as_float(sm.key[cur][pos] + rmin);
    }
    __syncthreads();
  }
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

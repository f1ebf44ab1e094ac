// Exact K-S change-point scan of one series per workgroup (gfx950).
//
// Per series (one workgroup of NT threads, NT/64 waves):
//   1. stream the K x N uint32 samples once: per row sum r and sum r^2
//      (96-bit), and the running minimum (eq. 2 needs the minimum over the
//      whole 2-D array);
//   2. Q_i = sum r^2 - 2 m sum r + N m^2 = sum_j (r_ij - m)^2, exact;
//   3. LDS LSD radix sort of the K (Q_i, i) pairs, RB-bit digits, only as
//      many passes as Q's bit length needs; mark the ends of equal-key groups;
//   4. lattice walk: for each candidate c, U_c = max over group ends p of
//      |K i_c(p) - c (p + 1)| with i_c(p) = #{q <= p : row(q) < c}, one
//      candidate per lane stepping through the sorted positions (this is
//      max |i m - j n| with j = p + 1 - i, the D numerator);
//   5. exact argmax of U_c^2 / (c (K - c)), eq. 1 significance, FP64
//      Kolmogorov p-value of the winner only.
#pragma once

#include <type_traits>

#include "ks.h"
#include "ks_wave.hpp"

namespace ks {

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- LDS layout

template <int KMAX, int NT, int RB>
struct ScanShape {
  static constexpr int W = NT / kWave;              // waves per workgroup
  static constexpr int T = (KMAX + NT - 1) / NT;    // sort tiles
  static constexpr int D = 1 << RB;                 // radix buckets
  static constexpr int H = D * T * W;               // (digit, tile, wave) counters
  static constexpr int CH = (KMAX + kWave - 1) / kWave;  // 64-position chunks
};

template <int KMAX, int NT, int RB>
struct ScanSmem {
  using S = ScanShape<KMAX, NT, RB>;
  union {
    struct {  // phase 1: per-row moments
      uint64_t s1[KMAX];
      uint64_t s2lo[KMAX];
      uint32_t s2hi[KMAX];
    } mom;
    struct {  // sort pong buffer (moments are dead once the keys exist)
      uint32_t key[3][KMAX];
      uint16_t idx[KMAX];
    } pong;
  } u;
  uint32_t key[3][KMAX];  // sort ping buffer: Q as three 32-bit words
  uint16_t idx[KMAX];
  uint64_t tie[S::CH];    // bit p%64 of tie[p/64]: sorted position p ends a group of equal Q
  uint16_t hist[S::H];
  uint32_t red[S::W * 4];
  uint32_t bestU[S::W], bestC[S::W];
  uint32_t partU[S::W * kWave];  // per-lane partial U_c of walks split over positions
};

// Moments of one row kept in device memory (split series of the persistent
// plan; every row of a series under binary segmentation, with the row's
// minimum in `pad`). 24 bytes.
struct RowMom {
  uint64_t s1;
  uint64_t s2lo;
  uint32_t s2hi;
  uint32_t pad;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ void acc_sample(uint32_t x, uint32_t& mn, uint64_t& s1, uint64_t& s2, uint32_t& s2h) {
  mn = min(mn, x);
  s1 += x;
  const uint64_t p = (uint64_t)x * x;
  s2 += p;
  s2h += (uint32_t)(s2 < p);
}

__device__ __forceinline__ uint32_t key_digit(uint32_t k0, uint32_t k1, uint32_t k2, int shift, uint32_t mask) {
  const int w = shift >> 5, o = shift & 31;
  const uint32_t a = w == 0 ? k0 : (w == 1 ? k1 : k2);
  const uint32_t b = w == 0 ? k1 : (w == 1 ? k2 : 0u);
  return (uint32_t)((((uint64_t)b << 32) | a) >> o) & mask;
}

// Does candidate a beat candidate b? lambda^2 = U^2 / (c (K - c) K); compared
// exactly by cross-multiplying (U^2 <= 2^40, c (K - c) <= 2^20).
__device__ __forceinline__ bool more_significant(uint32_t Ua, uint32_t a, uint32_t Ub, uint32_t b, uint32_t K) {
  const uint64_t lhs = (uint64_t)Ua * Ua * ((uint64_t)b * (K - b));
  const uint64_t rhs = (uint64_t)Ub * Ub * ((uint64_t)a * (K - a));
  return lhs > rhs || (lhs == rhs && a < b);
}

// Asymptotic Kolmogorov tail from lambda^2: the alternating exp(-2 k^2 l^2)
// series for lambda >= 1, the Jacobi-theta form below; each stops once a term
// is under 1e-20 of the sum; 0 once 2 lambda^2 > 700.
__device__ __noinline__ double kolmogorov_q(double lambda2) {
  if (!(lambda2 > 0.0)) return 1.0;
  if (2.0 * lambda2 > 700.0) return 0.0;
  double sum = 0.0;
  if (lambda2 >= 1.0) {
    for (int k = 1; k <= 200; ++k) {
      const double term = exp(-2.0 * lambda2 * (double)(k * k));
      sum += (k & 1) ? term : -term;
      if (term < 1e-20 * fabs(sum)) break;
    }
    return 2.0 * sum;
  }
  const double pi = 3.141592653589793;
  const double lam = sqrt(lambda2);
  for (int k = 1; k <= 200; ++k) {
    const double o = (double)(2 * k - 1);
    const double term = exp(-(o * o * pi * pi) / (8.0 * lambda2));
    sum += term;
    if (term < 1e-20 * sum) break;
  }
  return 1.0 - sqrt(2.0 * pi) / lam * sum;
}

__device__ __forceinline__ void write_result(ks_result* o, uint32_t cp, uint32_t n, uint32_t m, uint32_t U, double D,
                                             double lam, double p, uint32_t flags) {
  o->cp = cp;
  o->n = n;
  o->m = m;
  o->U = U;
  o->D = D;
  o->lambda = lam;
  o->p = p;
  o->flags = flags;
  o->pad = 0;
}

// ---------------------------------------------------------------- phases

// ---------------------------------------------------------------- streaming
//
// A wave streams its rows in batches: per lane up to four 16-byte loads of the
// row's 16-byte-aligned body (1024 samples per wave-batch), plus, in a row's
// last batch, one dword of the unaligned head or tail (lanes 0..2 / 32..34).
// The next batch is loaded before the current one is accumulated, so one
// batch per wave stays in flight while the wave computes; a row's sums are
// reduced with DPP once its last batch is in.

struct RowGeo {
  uint64_t e0;    // first sample of the row (element index from `samples`)
  uint32_t head;  // samples before the first 16-byte boundary
  uint32_t nq;    // 16-byte quads of the aligned body
  uint32_t tail;  // samples after the body
  uint32_t nb;    // batches (>= 1)
};

__device__ __forceinline__ RowGeo row_geo(const uint32_t* samples, uint64_t e0, uint32_t N) {
  RowGeo g;
  g.e0 = e0;
  const uint32_t a = (uint32_t)(((uintptr_t)(samples + e0) >> 2) & 3u);
  g.head = a ? min(4u - a, N) : 0u;
  g.nq = (N - g.head) >> 2;
  g.tail = (N - g.head) & 3u;
  g.nb = g.nq ? (g.nq + 4 * kWave - 1) / (4 * kWave) : 1u;
  return g;
}

struct Batch {
  u32x4 q[4];
  uint32_t x;
  uint32_t m;  // bit u: q[u] holds data; bit 4: x holds data
};

__device__ __forceinline__ void load_batch(Batch& B, const uint32_t* __restrict__ samples, const RowGeo& g,
                                           uint32_t b, uint32_t lane) {
  const u32x4* body = reinterpret_cast<const u32x4*>(samples + g.e0 + g.head);
  const uint32_t q0 = b * (4 * kWave) + lane;
  uint32_t m = 0;
  if (b * (4 * kWave) + 4 * kWave <= g.nq) {  // full batch (wave-uniform)
#pragma unroll
    for (int u = 0; u < 4; ++u) B.q[u] = __builtin_nontemporal_load(body + q0 + u * kWave);
    m = 15u;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (q0 + u * kWave < g.nq) {
        B.q[u] = __builtin_nontemporal_load(body + q0 + u * kWave);
        m |= 1u << u;
      } else {
        B.q[u] = u32x4{0u, 0u, 0u, 0u};
      }
    }
  }
  B.x = 0;
  // the head and tail samples share their 128-byte lines with the neighbouring
  // rows, which other waves read at about the same time: plain loads let the
  // L2 keep those lines for them (1% faster on a batch of uneven unaligned
  // rows; plain loads of the body quads as well were slower)
  if (b + 1 == g.nb) {
    if (lane < g.head) {
      B.x = samples[g.e0 + lane];
      m |= 16u;
    } else if (lane >= 32 && lane - 32 < g.tail) {
      B.x = samples[g.e0 + g.head + 4ull * g.nq + (lane - 32)];
      m |= 16u;
    }
  }
  B.m = m;
}

__device__ __forceinline__ void acc_quad(const u32x4& v, uint32_t& mn, uint64_t& s1, uint64_t& s2, uint32_t& s2h) {
  acc_sample(v.x, mn, s1, s2, s2h);
  acc_sample(v.y, mn, s1, s2, s2h);
  acc_sample(v.z, mn, s1, s2, s2h);
  acc_sample(v.w, mn, s1, s2, s2h);
}

__device__ __forceinline__ void acc_batch(const Batch& B, uint32_t& mn, uint64_t& s1, uint64_t& s2, uint32_t& s2h) {
  if ((B.m & 15u) == 15u) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc_quad(B.q[u], mn, s1, s2, s2h);
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (B.m & (1u << u)) acc_quad(B.q[u], mn, s1, s2, s2h);
  }
  if (B.m & 16u) acc_sample(B.x, mn, s1, s2, s2h);
}

// ---- short rows: several rows per wave
//
// A row of N <= 16 GL samples fits one batch of a GL-lane group (GL = 16: a
// DPP row of the wave; GL = 32: two), so a wave streams 64 / GL rows per step
// and each row's sums need only in-group DPP steps.

// Group sums: afterwards every lane of a 16-lane DPP row holds its row's
// total (GL = 16), or the upper row of each pair holds the pair's (GL = 32).
template <int GL>
__device__ __forceinline__ void group_total_64_96(uint64_t& s1, uint64_t& s2, uint32_t& s2h) {
  dpp_add64<kDppXor1>(s1);
  dpp_add96<kDppXor1>(s2, s2h);
  dpp_add64<kDppXor2>(s1);
  dpp_add96<kDppXor2>(s2, s2h);
  dpp_add64<kDppHalfMirror>(s1);
  dpp_add96<kDppHalfMirror>(s2, s2h);
  dpp_add64<kDppMirror>(s1);
  dpp_add96<kDppMirror>(s2, s2h);
  if constexpr (GL == 32) {
    dpp_add64<kDppBcast15, 0xA>(s1);
    dpp_add96<kDppBcast15, 0xA>(s2, s2h);
  }
}

template <int GL>
__device__ __forceinline__ uint32_t group_min_u32(uint32_t v) {
  v = min(v, dpp<kDppXor1>(v));
  v = min(v, dpp<kDppXor2>(v));
  v = min(v, dpp<kDppHalfMirror>(v));
  v = min(v, dpp<kDppMirror>(v));
  if constexpr (GL == 32)
    v = min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, kDppBcast15, 0xA, 0xF, false));
  return v;
}

// The group's row (when `valid`): the unaligned head in lanes 0.., the
// aligned body as 16-byte quads gl, gl + GL, ... (nqu of them at most, a
// wave-uniform bound), the tail in lanes GL / 2.. ; the rest zero.
template <int GL>
__device__ __forceinline__ void load_group(Batch& B, const uint32_t* __restrict__ samples, uint64_t e0, uint32_t N,
                                           bool valid, uint32_t gl, uint32_t nqu) {
  uint32_t m = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) B.q[u] = u32x4{0u, 0u, 0u, 0u};
  B.x = 0;
  if (valid) {
    const uint32_t a = (uint32_t)(((uintptr_t)(samples + e0) >> 2) & 3u);
    const uint32_t head = a ? min(4u - a, N) : 0u;
    const uint32_t nq = (N - head) >> 2, tail = (N - head) & 3u;
    const u32x4* body = reinterpret_cast<const u32x4*>(samples + e0 + head);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if ((uint32_t)u < nqu && gl + u * GL < nq) {
        B.q[u] = __builtin_nontemporal_load(body + gl + u * GL);
        m |= 1u << u;
      }
    }
    if (gl < head) {  // head and tail: plain loads, as in load_batch
      B.x = samples[e0 + gl];
      m |= 16u;
    } else if (gl >= GL / 2 && gl - GL / 2 < tail) {
      B.x = samples[e0 + head + 4ull * nq + (gl - GL / 2)];
      m |= 16u;
    }
  }
  B.m = m;
}

template <int GL, bool ROW_MIN, typename Emit>
__device__ __forceinline__ uint32_t stream_rows_grouped(const uint32_t* __restrict__ samples, uint64_t off,
                                                        uint32_t N, uint32_t rb, uint32_t re, uint32_t step,
                                                        uint32_t lane, Emit&& emit) {
  constexpr uint32_t RPW = kWave / GL;  // rows per wave step
  uint32_t mn = 0xffffffffu;
  if (rb >= re) return mn;
  const uint32_t g = lane / GL, gl = lane % GL;
  const uint32_t nqu = min(4u, ((N >> 2) + GL - 1) / GL);
  // step i, group g: row rb + (i RPW + g) step. One batch of registers: the
  // next rows' loads go out once this step's samples are summed, ahead of
  // the group reductions and the emits.
  uint32_t base = rb;
  Batch cur;
  {
    const uint32_t row = base + g * step;
    load_group<GL>(cur, samples, off + (uint64_t)row * N, N, row < re, gl, nqu);
  }
  for (;;) {
    uint64_t s1 = 0, s2 = 0;
    uint32_t s2h = 0, rmn = 0xffffffffu;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if ((uint32_t)u < nqu && (cur.m & (1u << u))) acc_quad(cur.q[u], ROW_MIN ? rmn : mn, s1, s2, s2h);
    if (cur.m & 16u) acc_sample(cur.x, ROW_MIN ? rmn : mn, s1, s2, s2h);
    const uint32_t nbase = base + RPW * step;
    const bool more = nbase < re;
    if (more) {
      const uint32_t row = nbase + g * step;
      load_group<GL>(cur, samples, off + (uint64_t)row * N, N, row < re, gl, nqu);
    }
    group_total_64_96<GL>(s1, s2, s2h);
    if constexpr (ROW_MIN) {
      rmn = group_min_u32<GL>(rmn);
      mn = min(mn, rmn);
    }
#pragma unroll
    for (uint32_t gg = 0; gg < RPW; ++gg) {
      const uint32_t row = base + gg * step;
      if (row < re) {
        const int src = (int)(gg * GL + GL - 1);
        const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s1, src);
        const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(s1 >> 32), src);
        const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s2, src);
        const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(s2 >> 32), src);
        const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)s2h, src);
        const uint32_t rm = ROW_MIN ? (uint32_t)__builtin_amdgcn_readlane((int)rmn, src) : 0xffffffffu;
        emit(row, ((uint64_t)b << 32) | a, ((uint64_t)d << 32) | c, h, rm);
      }
    }
    if (!more) break;
    base = nbase;
  }
  return mn;
}

// Streams rows rb, rb + step, ... < re of the series whose row i starts at
// samples[off + i N]. For each row, emit(i, s1, s2lo, s2hi, row_min) receives
// the wave-uniform totals (sum r, sum r^2) and, when ROW_MIN, the row's
// minimum (0xffffffff otherwise). Returns this lane's running minimum. Rows
// of up to 512 samples go several to a wave (stream_rows_grouped).
template <bool ROW_MIN = false, typename Emit>
__device__ __forceinline__ uint32_t stream_rows(const uint32_t* __restrict__ samples, uint64_t off, uint32_t N,
                                                uint32_t rb, uint32_t re, uint32_t step, uint32_t lane,
                                                Emit&& emit) {
  if (N <= 16u * 16u) return stream_rows_grouped<16, ROW_MIN>(samples, off, N, rb, re, step, lane, emit);
  if (N <= 16u * 32u) return stream_rows_grouped<32, ROW_MIN>(samples, off, N, rb, re, step, lane, emit);
  uint32_t mn = 0xffffffffu;
  if (rb >= re) return mn;
  uint32_t rmn = 0xffffffffu;  // this row's lane minimum (ROW_MIN)
  uint32_t row = rb, b = 0;
  RowGeo g = row_geo(samples, off + (uint64_t)row * N, N);
  Batch cur, nxt;
  load_batch(cur, samples, g, 0, lane);
  uint64_t s1 = 0, s2 = 0;
  uint32_t s2h = 0;
  for (;;) {
    uint32_t nrow = row, nbb = b + 1;
    RowGeo ng = g;
    if (nbb == g.nb) {
      nrow = row + step;
      nbb = 0;
      if (nrow < re) ng = row_geo(samples, off + (uint64_t)nrow * N, N);
    }
    const bool more = nrow < re;
    if (more) load_batch(nxt, samples, ng, nbb, lane);
    acc_batch(cur, ROW_MIN ? rmn : mn, s1, s2, s2h);
    if (b + 1 == g.nb) {
      wave_total_64_96(s1, s2, s2h);
      uint32_t row_min = 0xffffffffu;
      if constexpr (ROW_MIN) {
        row_min = wave_min_u32(rmn);
        mn = min(mn, row_min);
        rmn = 0xffffffffu;
      }
      emit(row, s1, s2, s2h, row_min);
      s1 = 0;
      s2 = 0;
      s2h = 0;
    }
    if (!more) break;
    cur = nxt;
    row = nrow;
    b = nbb;
    g = ng;
  }
  return mn;
}

// Block-wide minimum of a per-lane value (all threads get it).
template <int NT>
__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t* red) {
  constexpr int W = NT / kWave;
  const uint32_t lane = lane_id(), w = wave_id();
  v = wave_min_u32(v);
  if (lane == 0) red[w] = v;
  __syncthreads();
  uint32_t g = red[0];
#pragma unroll
  for (int k = 1; k < W; ++k) g = min(g, red[k]);
  __syncthreads();
  return g;
}

// Phase 1: per-row moments into LDS; returns the series minimum (block-uniform).
template <int KMAX, int NT, int RB>
__device__ uint32_t stream_moments(ScanSmem<KMAX, NT, RB>& sm, const uint32_t* __restrict__ samples, uint64_t off,
                                   uint32_t K, uint32_t N) {
  using S = ScanShape<KMAX, NT, RB>;
  const uint32_t lane = lane_id(), w = wave_id();
  const uint32_t mn = stream_rows(samples, off, N, w, K, S::W, lane,
                                  [&](uint32_t i, uint64_t s1, uint64_t s2, uint32_t s2h, uint32_t) {
                                    if (lane == 0) {
                                      sm.u.mom.s1[i] = s1;
                                      sm.u.mom.s2lo[i] = s2;
                                      sm.u.mom.s2hi[i] = s2h;
                                    }
                                  });
  return block_min_u32<NT>(mn, sm.red);
}

// Phase 2: Q_i keys (ping buffer) and their OR (for the number of radix passes).
template <int KMAX, int NT, int RB>
__device__ int make_keys(ScanSmem<KMAX, NT, RB>& sm, uint32_t K, uint32_t N, uint32_t gmin) {
  using S = ScanShape<KMAX, NT, RB>;
  const uint32_t lane = lane_id(), w = wave_id();
  uint32_t o0 = 0, o1 = 0, o2 = 0;
  const u128 nm2 = (u128)((uint64_t)gmin * gmin) * N;
  const uint64_t twom = 2ull * gmin;
  for (uint32_t i = threadIdx.x; i < K; i += NT) {
    const u128 s2 = ((u128)sm.u.mom.s2hi[i] << 64) | sm.u.mom.s2lo[i];
    const u128 q = s2 + nm2 - (u128)sm.u.mom.s1[i] * twom;
    const uint32_t k0 = (uint32_t)q, k1 = (uint32_t)(q >> 32), k2 = (uint32_t)(q >> 64);
    sm.key[0][i] = k0;
    sm.key[1][i] = k1;
    sm.key[2][i] = k2;
    sm.idx[i] = (uint16_t)i;
    o0 |= k0;
    o1 |= k1;
    o2 |= k2;
  }
  o0 = wave_or_u32(o0);
  o1 = wave_or_u32(o1);
  o2 = wave_or_u32(o2);
  if (lane == 0) {
    sm.red[w * 4 + 0] = o0;
    sm.red[w * 4 + 1] = o1;
    sm.red[w * 4 + 2] = o2;
  }
  __syncthreads();
  uint32_t a = 0, b = 0, c = 0;
#pragma unroll
  for (int v = 0; v < S::W; ++v) {
    a |= sm.red[v * 4 + 0];
    b |= sm.red[v * 4 + 1];
    c |= sm.red[v * 4 + 2];
  }
  __syncthreads();
  if (c) return 96 - __clz(c);
  if (b) return 64 - __clz(b);
  if (a) return 32 - __clz(a);
  return 0;
}

// Phase 3: stable LSD radix sort of (key, idx); returns true if the sorted
// data ended in the pong buffer.
template <int KMAX, int NT, int RB>
__device__ bool sort_keys(ScanSmem<KMAX, NT, RB>& sm, uint32_t K, int bits) {
  using S = ScanShape<KMAX, NT, RB>;
  const uint32_t lane = lane_id(), w = wave_id(), tid = threadIdx.x;
  const int passes = (bits + RB - 1) / RB;
  constexpr int C = (S::H + NT - 1) / NT;
  for (int p = 0; p < passes; ++p) {
    const bool from_ping = (p & 1) == 0;
    uint32_t(*ka)[KMAX] = from_ping ? sm.key : sm.u.pong.key;
    uint16_t* ia = from_ping ? sm.idx : sm.u.pong.idx;
    uint32_t(*kb)[KMAX] = from_ping ? sm.u.pong.key : sm.key;
    uint16_t* ib = from_ping ? sm.u.pong.idx : sm.idx;
    const int shift = p * RB;
    for (int h = tid; h < S::H; h += NT) sm.hist[h] = 0;
    __syncthreads();
    uint32_t dg[S::T], rk[S::T];
#pragma unroll
    for (int t = 0; t < S::T; ++t) {
      const uint32_t item = t * NT + tid;
      const bool valid = item < K;
      const uint32_t d = valid ? key_digit(ka[0][item], ka[1][item], ka[2][item], shift, S::D - 1) : 0u;
      uint64_t peers = ballot(valid);
#pragma unroll
      for (int b = 0; b < RB; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
      }
      dg[t] = d;
      rk[t] = mbcnt(peers);
      if (valid && rk[t] == 0) sm.hist[(d * S::T + t) * S::W + w] = (uint16_t)__popcll(peers);
    }
    __syncthreads();
    // exclusive scan of hist in (digit, tile, wave) order
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
    for (uint32_t v = 0; v < w; ++v) run += sm.red[v];
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
    for (int t = 0; t < S::T; ++t) {
      const uint32_t item = t * NT + tid;
      if (item < K) {
        const uint32_t dst = sm.hist[(dg[t] * S::T + t) * S::W + w] + rk[t];
        kb[0][dst] = ka[0][item];
        kb[1][dst] = ka[1][item];
        kb[2][dst] = ka[2][item];
        ib[dst] = ia[item];
      }
    }
    __syncthreads();
  }
  return (passes & 1) != 0;
}

// ---------------------------------------------------------------- lattice walk
//
// The candidate sits on the lane: lane l of slot j holds c = c_lo + 64 j + l
// and D_c(p) = K i_c(p) - c (p + 1), i_c(p) = #{q <= p : row(q) < c}, for the
// sorted positions p in order. Each step adds K - c where the row at p is
// below c and -c otherwise (the row is the same for every lane, read once per
// four positions); U_c = max over tie-group ends of |D_c(p)| is kept as a
// running max and min of D. No cross-lane work until the argmax at the end.

// |D| <= c (K - c) <= K^2 / 4 < 2^21: int32 holds every step.
template <int G>
__device__ __forceinline__ void walk_step(uint32_t r, const uint32_t (&c)[G], const int32_t (&up)[G],
                                          const int32_t (&dn)[G], int32_t (&D)[G]) {
#pragma unroll
  for (int g = 0; g < G; ++g) D[g] += r < c[g] ? up[g] : dn[g];
}

// Positions [pa, pb) of one pass. TIES = false: every position ends a group
// (no two Q equal), so the walk takes eight positions per broadcast read with
// no per-position test; TIES = true reads the group-end bits.
template <int KMAX, int G, bool TIES>
__device__ __forceinline__ void walk_positions(const uint16_t* __restrict__ is, const uint64_t* __restrict__ tie,
                                               uint32_t pa, uint32_t pb, uint32_t K, const uint32_t (&c)[G],
                                               int32_t (&D)[G], int32_t (&mx)[G], int32_t (&mn)[G]) {
  int32_t up[G], dn[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    up[g] = (int32_t)K - (int32_t)c[g];
    dn[g] = -(int32_t)c[g];
  }
  uint32_t p = pa;
  if constexpr (!TIES) {
    // pa is a multiple of 8: two 8-byte aligned broadcast reads per group,
    // the next group's issued before this one's arithmetic (the address
    // clamped inside the KMAX-entry array; a clamped read goes unused)
    uint2 na = make_uint2(0u, 0u), nb = make_uint2(0u, 0u);
    if (p + 8 <= pb) {
      na = *reinterpret_cast<const uint2*>(is + p);
      nb = *reinterpret_cast<const uint2*>(is + p + 4);
    }
    for (; p + 8 <= pb; p += 8) {
      const uint2 ra = na, rb = nb;
      const uint32_t pn = min(p + 8, KMAX - 8u);
      na = *reinterpret_cast<const uint2*>(is + pn);
      nb = *reinterpret_cast<const uint2*>(is + pn + 4);
      const uint32_t w[4] = {(uint32_t)__builtin_amdgcn_readfirstlane((int)ra.x),
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)ra.y),
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)rb.x),
                             (uint32_t)__builtin_amdgcn_readfirstlane((int)rb.y)};
#pragma unroll
      for (int g = 0; g < G; ++g) {
        int32_t v[8];
        int32_t x = D[g];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const uint32_t r = (j & 1) ? (w[j >> 1] >> 16) : (w[j >> 1] & 0xffffu);
          x += r < c[g] ? up[g] : dn[g];
          v[j] = x;
        }
#pragma unroll
        for (int j = 0; j < 8; j += 2) {
          mx[g] = max(max(mx[g], v[j]), v[j + 1]);
          mn[g] = min(min(mn[g], v[j]), v[j + 1]);
        }
        D[g] = x;
      }
    }
  }
  // the rest one position at a time (TIES: all of [pa, pb))
  for (; p < pb; ++p) {
    const uint32_t r = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)is[p]);
    walk_step<G>(r, c, up, dn, D);
    bool end = true;
    if constexpr (TIES) {
      const uint64_t t = tie[p >> 6] >> (p & 63);
      end = (__builtin_amdgcn_readfirstlane((int)(uint32_t)t) & 1) != 0;
    }
    if (end) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        mx[g] = max(mx[g], D[g]);
        mn[g] = min(mn[g], D[g]);
      }
    }
  }
}

// Best (U, c) of a wave: exact lambda order, ties to the smaller c; c = 0 is
// "no candidate". A float key U^2 / (c (K - c)) (relative error under 2^-21:
// U^2 rounded once, an rcp within 1 ulp, one rounded product) finds the
// maximum by a DPP max; every lane within 16 ulps of it (2^-20 relative or
// more) is then compared exactly, one lane at a time.
__device__ __forceinline__ void wave_best(uint32_t& U, uint32_t& c, uint32_t K) {
  uint32_t key = 0;
  if (c != 0) {
    const float u = (float)U;  // U <= K^2 / 4 < 2^24: exact
    const float f = (u * u) * __builtin_amdgcn_rcpf((float)(c * (K - c)));
    key = __float_as_uint(f) + 1u;  // f >= 0: bits order as f; 0 stays "none"
  }
  const uint32_t kmax = wave_max_u32(key);
  uint64_t cand = ballot(key != 0 && key + 16u >= kmax);
  uint32_t bu = 0, bc = 0;
  while (cand) {
    const int l = __builtin_ctzll(cand);
    cand &= cand - 1;
    const uint32_t u = (uint32_t)__builtin_amdgcn_readlane((int)U, l);
    const uint32_t cc = (uint32_t)__builtin_amdgcn_readlane((int)c, l);
    if (bc == 0 || more_significant(u, cc, bu, bc, K)) {
      bu = u;
      bc = cc;
    }
  }
  U = bu;
  c = bc;
}

// Walk of one pass over G slots (wave-uniform) on positions [pa, pb); with
// pa > 0, D starts from K i_c(pa - 1) - c pa, the count taken from pos[]
// (the sorted position of every row). Returns the partial U per slot.
template <int KMAX, int G>
__device__ __forceinline__ void walk_pass(const uint16_t* __restrict__ is, const uint16_t* __restrict__ pos,
                                          const uint64_t* __restrict__ tie, bool ties, uint32_t K, uint32_t pa,
                                          uint32_t pb, const uint32_t (&c)[G], uint32_t (&U)[G]) {
  const uint32_t lane = lane_id();
  int32_t D[G], mx[G], mn[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    D[g] = 0;
    mx[g] = 0;  // D = 0 at p = K - 1 (always a group end): 0 bounds U from below
    mn[g] = 0;
  }
  if (pa > 0) {
    uint32_t cnt[G];
#pragma unroll
    for (int g = 0; g < G; ++g) cnt[g] = 0;
    for (uint32_t j = 0; j * kWave < K; ++j) {
      const uint32_t r = j * kWave + lane;
      const uint64_t bal = ballot(r < K && pos[r] < pa);
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int32_t x = (int32_t)c[g] - (int32_t)(j * kWave);  // rows of this chunk below c
        const uint64_t m = x >= kWave ? ~0ull : (x <= 0 ? 0ull : ((1ull << x) - 1ull));
        cnt[g] += (uint32_t)__popcll(bal & m);
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) D[g] = (int32_t)(K * cnt[g]) - (int32_t)(c[g] * pa);
  }
  if (ties)
    walk_positions<KMAX, G, true>(is, tie, pa, pb, K, c, D, mx, mn);
  else
    walk_positions<KMAX, G, false>(is, tie, pa, pb, K, c, D, mx, mn);
#pragma unroll
  for (int g = 0; g < G; ++g) U[g] = (uint32_t)max(mx[g], -mn[g]);
}

// Candidates c_lo..c_hi over 64-lane slots. With at least one slot per wave,
// wave w walks every position for slots w, w + W, ... (up to kMaxG at a time);
// with fewer slots than waves, the waves of a slot split the positions (shares
// of a multiple of 8) and their partial maxima meet in LDS. ties: some two Q
// are equal. (bU, bC) is the wave's best (bC = 0: none).
template <int KMAX, int NT, int RB, int GM = 0>
__device__ void walk_splits(ScanSmem<KMAX, NT, RB>& sm, const uint16_t* __restrict__ is, uint16_t* __restrict__ pos,
                            bool ties, uint32_t K, uint32_t c_lo, uint32_t c_hi, uint32_t* __restrict__ allU,
                            uint32_t& bU, uint32_t& bC) {
  using S = ScanShape<KMAX, NT, RB>;
  constexpr int W = S::W;
  // slots a wave walks at once: as many as its share (at most 4), or at most GM when GM > 0
  constexpr int kShareG = S::CH / W < 1 ? 1 : (S::CH / W > 4 ? 4 : S::CH / W);
  constexpr int kMaxG = GM > 0 && GM < kShareG ? GM : kShareG;
  const uint32_t lane = lane_id(), w = wave_id();
  const uint32_t n = c_hi >= c_lo ? c_hi - c_lo + 1 : 0;
  const uint32_t ns = (n + kWave - 1) / kWave;
  bU = 0;
  bC = 0;
  auto consider = [&](uint32_t c, uint32_t U) {
    if (c > c_hi) return;
    if (allU) allU[c] = U;
    if (bC == 0 || more_significant(U, c, bU, bC, K)) {
      bU = U;
      bC = c;
    }
  };
  if (ns >= (uint32_t)W) {
    const uint32_t mine = ns / W + (w < ns % W ? 1u : 0u);  // slots w, w + W, ...
    for (uint32_t j0 = 0; j0 < mine;) {
      const uint32_t take = min(mine - j0, (uint32_t)kMaxG);
      auto run = [&](auto gtag) {
        constexpr int G = decltype(gtag)::value;
        uint32_t c[G], U[G];
#pragma unroll
        for (int g = 0; g < G; ++g) c[g] = c_lo + (w + (j0 + g) * W) * kWave + lane;
        walk_pass<KMAX, G>(is, nullptr, sm.tie, ties, K, 0, K, c, U);
#pragma unroll
        for (int g = 0; g < G; ++g) consider(c[g], U[g]);
      };
      if (take == 4) run(std::integral_constant<int, (kMaxG >= 4 ? 4 : 1)>{});
      else if (take == 3) run(std::integral_constant<int, (kMaxG >= 3 ? 3 : 1)>{});
      else if (take == 2) run(std::integral_constant<int, (kMaxG >= 2 ? 2 : 1)>{});
      else run(std::integral_constant<int, 1>{});
      j0 += take;
    }
  } else if (ns > 0) {
    // fewer slots than waves: P waves per slot, each a 4-aligned share of the positions
    const uint32_t P = W / ns;
    const uint32_t slot = w / P, part = w % P;
    for (uint32_t p = threadIdx.x; p < K; p += NT) pos[is[p]] = (uint16_t)p;
    __syncthreads();
    const uint32_t len = ((K + P - 1) / P + 7u) & ~7u;
    uint32_t c[1], U[1] = {0};
    c[0] = c_lo + slot * kWave + lane;
    if (slot < ns) {
      const uint32_t pa = min(K, part * len), pb = min(K, pa + len);
      walk_pass<KMAX, 1>(is, pos, sm.tie, ties, K, pa, pb, c, U);
    }
    sm.partU[w * kWave + lane] = U[0];
    __syncthreads();
    if (slot < ns && part == 0) {
      for (uint32_t q = 1; q < P; ++q) U[0] = max(U[0], sm.partU[(w + q) * kWave + lane]);
      consider(c[0], U[0]);
    }
  }
  wave_best(bU, bC, K);
}

// Phases 4-5 for one series already holding moments in LDS: the walk and the
// choice cover the candidates c_lo..c_hi (inclusive; 1..K-1 for the full
// scan); extra_flags are or-ed into the result flags.
template <int KMAX, int NT, int RB, int GM = 0>
__device__ void finish_series(ScanSmem<KMAX, NT, RB>& sm, uint32_t K, uint32_t N, uint32_t gmin,
                              const ks_params& prm, ks_result* __restrict__ out, uint32_t* __restrict__ allU,
                              uint32_t c_lo = 1, uint32_t c_hi = 0xffffffffu, uint32_t extra_flags = 0) {
  if (c_hi > K - 1) c_hi = K - 1;
  if (c_lo < 1) c_lo = 1;
  using S = ScanShape<KMAX, NT, RB>;
  const uint32_t lane = lane_id(), w = wave_id();
  const int bits = make_keys(sm, K, N, gmin);
  const bool in_pong = sort_keys(sm, K, bits);
  uint32_t(*ks)[KMAX] = in_pong ? sm.u.pong.key : sm.key;
  const uint16_t* is = in_pong ? sm.u.pong.idx : sm.idx;

  // ends of equal-key groups
  bool any_tie = false;
  for (uint32_t p0 = w * kWave; p0 < K; p0 += NT) {
    const uint32_t p = p0 + lane;
    bool end = false;
    if (p + 1 < K)
      end = ks[0][p] != ks[0][p + 1] || ks[1][p] != ks[1][p + 1] || ks[2][p] != ks[2][p + 1];
    else if (p + 1 == K)
      end = true;
    const uint64_t m = ballot(end);
    if (lane == 0) sm.tie[p0 / kWave] = m;
    any_tie |= m != ballot(p < K);
  }
  if (lane == 0) sm.red[w] = any_tie ? 1u : 0u;
  __syncthreads();
  bool ties = false;
#pragma unroll
  for (int v = 0; v < S::W; ++v) ties |= sm.red[v] != 0;

  uint32_t bU = 0, bC = 0;
  walk_splits<KMAX, NT, RB, GM>(sm, is, in_pong ? sm.idx : sm.u.pong.idx, ties, K, c_lo, c_hi, allU, bU, bC);
  if (lane == 0) {
    sm.bestU[w] = bU;
    sm.bestC[w] = bC;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t U = sm.bestU[0], c = sm.bestC[0];
    for (int v = 1; v < S::W; ++v)
      if (sm.bestC[v] != 0 && (c == 0 || more_significant(sm.bestU[v], sm.bestC[v], U, c, K))) {
        U = sm.bestU[v];
        c = sm.bestC[v];
      }
    if (allU) allU[0] = 0;
    if (c == 0) {  // empty range (not reached by the callers)
      c = c_lo;
      U = 0;
    }
    const uint32_t n = c, m = K - c;
    const double U2 = (double)((uint64_t)U * U);
    const double nmK = (double)((uint64_t)n * m * K);
    const double lambda2 = U2 / nmK;
    const double p = U == 0 ? 1.0 : kolmogorov_q(lambda2);
    const uint32_t flags = ((U2 > prm.c_alpha * nmK) ? KS_SIGNIFICANT : 0u) | extra_flags;
    write_result(out, c, n, m, U, (double)U / (double)((uint64_t)n * m), sqrt(lambda2), p, flags);
  }
  __syncthreads();
}

// Shape / range validation of one descriptor (uniform across the workgroup).
__device__ __forceinline__ uint32_t check_desc(const ks_desc& d, uint64_t num_samples, uint32_t max_K) {
  if (d.K < 2 || d.K > max_K || d.N < 1 || d.N > KS_MAX_N) return KS_BAD_SHAPE;
  if (d.offset > num_samples || (uint64_t)d.K * d.N > num_samples - d.offset) return KS_OUT_OF_RANGE;
  return 0;
}

template <int KMAX, int NT, int RB, int GM = 0>
__device__ void scan_one(ScanSmem<KMAX, NT, RB>& sm, const uint32_t* __restrict__ samples, uint64_t num_samples,
                         const ks_desc& d, const ks_params& prm, uint32_t max_K, ks_result* __restrict__ out,
                         uint32_t* __restrict__ allU, uint64_t allU_len) {
  const uint32_t bad = check_desc(d, num_samples, max_K);
  if (bad) {
    if (threadIdx.x == 0) write_result(out, 0, 0, 0, 0, 0.0, 0.0, 1.0, bad);
    return;
  }
  const uint32_t gmin = stream_moments(sm, samples, d.offset, d.K, d.N);
  const bool fits = allU && d.aux_offset <= allU_len && d.K <= allU_len - d.aux_offset;
  finish_series<KMAX, NT, RB, GM>(sm, d.K, d.N, gmin, prm, out, fits ? allU + d.aux_offset : nullptr);
}

// One workgroup per series; with `order`, workgroup b takes series order[b]
// (the plan's largest-first order, one item per series, 8-byte items whose
// first word is the series).
template <int KMAX, int NT, int RB, int GM = 0>
__global__ __launch_bounds__(NT) void scan_kernel(const uint32_t* __restrict__ samples, uint64_t num_samples,
                                                  const ks_desc* __restrict__ desc, uint32_t num_series,
                                                  ks_params prm, uint32_t max_K, ks_result* __restrict__ out,
                                                  uint32_t* __restrict__ allU, uint64_t allU_len,
                                                  const uint32_t* __restrict__ order) {
  __shared__ ScanSmem<KMAX, NT, RB> sm;
  if (blockIdx.x >= num_series) return;
  const uint32_t s = order ? __builtin_amdgcn_readfirstlane(order[2 * blockIdx.x]) : blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  scan_one<KMAX, NT, RB, GM>(sm, samples, num_samples, d, prm, max_K, out + s, allU, allU_len);
}

}  // namespace ks

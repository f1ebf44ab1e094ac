// Order statistics of rows of uint32 samples, one wave per row: the row held
// in registers (1, 2 or 4 load batches), its moments (sum r, sum r^2), minimum
// and maximum by DPP, and a multi-rank MSD radix select for up to nine target
// ranks. Used by the learned path's decile features and by the per-row
// latency statistics.
#pragma once

#include "ks_scan.hpp"
#include "ks_wave.hpp"

namespace ks {

// ------------------------------------------------------------------ deciles
// Up to nine order statistics of one row, found by one wave with no block
// barrier, over the keys r - row minimum.
//
// Window level. One histogram pass with one bin per key value below
// kSelWin - 1 and a last bin for every larger key: order statistics of latency
// rows sit in the bulk of the row, within a few hundred cycles of its minimum,
// so this single pass resolves them exactly (a target's value is its bin).
// The bins' counts are summed per lane (16 bins each), a wave scan gives each
// lane's base, a ballot per target finds the lane whose bins hold its rank,
// and that lane's 16 bins give the bin.
//
// Radix levels, for targets that fall into the last bin (and for rows whose
// keys may equal the empty-slot sentinel): an MSD radix select over the keys
// of that bin. Level 0 histograms the top kSelW0 bits of every key; each later
// level histograms the next kSelW bits of only the keys that share a target's
// prefix so far. Those keys form at most nine groups (one per distinct prefix
// among the targets), numbered in target order. After each level every key is
// rewritten in place as (group << s) | (its s low bits), s the bits still
// unresolved, with group kSelNone for keys outside every group, so the next
// level's bin is the key shifted right by the next s. Histograms are LDS
// counters per (group, digit) bin; keys whose bin lies past the live groups
// issue no LDS access (such keys would pile onto a few addresses and serialise
// the atomics).

constexpr uint32_t kSelWin = 1024; // bins of the window level: keys 0 .. 1022 one each, 1023 the rest
constexpr uint32_t kSelW0 = 10;    // bits of the level-0 digit (1024 bins fit the histogram)
constexpr uint32_t kSelW = 7;      // bits of every later digit
constexpr uint32_t kSelNone = 9;   // group of keys outside every target's prefix
constexpr uint32_t kSelEmpty = 0xffffffffu;  // key of a slot without a sample

struct __align__(16) SelLds {
  uint32_t hist[(kSelNone + 1) << kSelW];  // bin counts, then exclusive prefixes
  uint8_t tab[(kSelNone + 1) << kSelW];    // bin -> group at the next level
};
static_assert((1u << kSelW0) <= ((kSelNone + 1) << kSelW), "level-0 bins fit the histogram");
static_assert(kSelWin == 16u * kWave && kSelWin + kWave <= ((kSelNone + 1) << kSelW),
              "16 window bins per lane and a spare word per lane fit");
static_assert((((kSelNone << kSelW) + 255u) & ~255u) <= ((kSelNone + 1) << kSelW), "padded live bins fit");

// LDS accesses of one wave are performed in order; this keeps the compiler
// from moving them across the point where lanes exchange data through LDS.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exclusive prefix sums, in place, over hist[0, 256 nblk), bins in order. Lane
// l owns bins 256 i + 4 l .. 256 i + 4 l + 3 of block i, so every access is a
// conflict-free 16-byte one; two blocks share one wave scan, packed as 16-bit
// halves (a wave holds fewer than 2^16 keys, so no half carries into the next).
__device__ __forceinline__ void wave_excl_prefix(uint32_t* hist, uint32_t nblk, uint32_t lane) {
  uint32_t base = 0;
  for (uint32_t i = 0; i < nblk; i += 2) {
    const bool two = i + 1 < nblk;
    u32x4* pa = reinterpret_cast<u32x4*>(hist + 256u * i + 4u * lane);
    u32x4* pc = reinterpret_cast<u32x4*>(hist + 256u * (i + 1) + 4u * lane);
    const u32x4 a = *pa;
    const u32x4 c = two ? *pc : u32x4{0u, 0u, 0u, 0u};
    const uint32_t sa = a.x + a.y + a.z + a.w, sc = c.x + c.y + c.z + c.w;
    const uint32_t incl = wave_incl_scan(sa | (sc << 16));
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    const uint32_t ea = base + (incl & 0xffffu) - sa;
    const uint32_t basec = base + (tot & 0xffffu);
    const uint32_t ec = basec + (incl >> 16) - sc;
    *pa = u32x4{ea, ea + a.x, ea + a.x + a.y, ea + a.x + a.y + a.z};
    if (two) *pc = u32x4{ec, ec + c.x, ec + c.x + c.y, ec + c.x + c.y + c.z};
    base = basec + (tot >> 16);
  }
}

// Target ranks of a select: RANKS::kCount <= 9 targets, RANKS::rank(j, N)
// non-decreasing in j.
// The nine deciles x_(floor(k (N - 1) / 10)), k = 1..9.
struct DecileRanks {
  static constexpr uint32_t kCount = 9;
  __device__ static uint32_t rank(uint32_t j, uint32_t N) { return (uint32_t)(((uint64_t)(j + 1) * (N - 1)) / 10u); }
};

// Radix levels. k[]: this lane's keys, every one below 2^b (b >= 1), empty
// slots holding kSelEmpty, which lies past every level-0 bin unless b = 32,
// and then sorts at or after every key; the keys are consumed. Lanes with tl
// (at most kSelNone of them, consecutive lanes, ranks R non-decreasing with
// the lane) return the key of rank R.
template <int V>
__device__ __forceinline__ uint32_t radix_select(SelLds& L, uint32_t (&k)[V], uint32_t b, uint32_t R, bool tl,
                                                 uint32_t lane) {
  const uint64_t tm = ballot(tl);
  const uint32_t first = tm ? (uint32_t)__builtin_ctzll(tm) : 0u;  // participating lanes: first, first + 1, ...
  uint32_t tg = 0, key = 0, G = 1, sprev = b, wmax = kSelW0;
#pragma unroll 1
  for (;;) {
    const uint32_t w = min(sprev, wmax);
    const uint32_t s = sprev - w;
    const uint32_t nblk = ((G << w) + 255u) >> 8;  // 256-bin blocks covering groups 0..G-1
    for (uint32_t i = 0; i < nblk; ++i)
      *reinterpret_cast<u32x4*>(L.hist + 256u * i + 4u * lane) = u32x4{0u, 0u, 0u, 0u};
    wave_lds_sync();
    const uint32_t live = G << w;  // bins of groups 0..G-1; keys past them are not counted
#pragma unroll
    for (int e = 0; e < V; ++e) {
      const uint32_t x = k[e] >> s;
      if (x < live) atomicAdd(&L.hist[x], 1u);
      if (V > 17 && e % 17 == 16) __builtin_amdgcn_sched_barrier(0);  // bounds the addresses in flight
    }
    wave_lds_sync();
    wave_excl_prefix(L.hist, nblk, lane);
    wave_lds_sync();
    // each target: the last bin of its group whose prefix is <= its rank
    uint32_t x = 0;
    if (tl) {
      const uint32_t x0 = tg << w;
      const uint32_t Rg = L.hist[x0] + R;
      x = x0;
      for (uint32_t bit = w; bit-- > 0;) {
        const uint32_t y = x + (1u << bit);
        if (L.hist[y] <= Rg) x = y;
      }
      R = Rg - L.hist[x];
      key = (key << w) | (x - x0);
    }
    if (s == 0) break;
    // groups of the next level: the targets' distinct bins, in target order
    const uint32_t prev = (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    const bool fresh = tl && (lane == first || x != prev);
    const uint64_t m = ballot(fresh);
    const uint32_t id = mbcnt(m) - (fresh ? 0u : 1u);
    const uint32_t words = live / 4u;
    uint32_t* tw = reinterpret_cast<uint32_t*>(L.tab);
    for (uint32_t q = lane; q < words; q += kWave) tw[q] = kSelNone * 0x01010101u;
    wave_lds_sync();
    if (tl) L.tab[x] = (uint8_t)id;
    wave_lds_sync();
    // a fresh copy of s, so that the compiler recomputes each bin here rather
    // than keeping all of them live from the histogram loop
    uint32_t s2 = s;
    asm volatile("" : "+v"(s2));
    const uint32_t low = (1u << s) - 1u;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      // unconditional read at a clamped bin (reads of one address broadcast)
      const uint32_t x = k[e] >> s2;
      const uint32_t t = L.tab[min(x, live - 1u)];
      k[e] = ((x < live ? t : kSelNone) << s) | (k[e] & low);
      if (V > 17 && e % 17 == 16) __builtin_amdgcn_sched_barrier(0);  // bounds the lookups in flight
    }
    wave_lds_sync();
    tg = id;
    G = (uint32_t)__popcll(m);
    sprev = s;
    wmax = kSelW;
  }
  return key;
}

// key(e), e < V: this lane's keys (values - row minimum, empty slots
// kSelEmpty), computed on demand so that no key array stays live through the
// pass; b >= 1 the bit length of the row's range. Lane j < RANKS::kCount
// returns the key of rank RANKS::rank(j, N), N the number of keys in the wave.
// DENSE: only slots e with e % 17 == 16 can be empty (the head / tail slot of
// each full load batch), so the others skip the check.
template <int V, class RANKS, bool DENSE, class KeyFn>
__device__ __forceinline__ uint32_t wave_select_fn(SelLds& L, KeyFn&& keyf, uint32_t b, uint32_t N, uint32_t lane) {
  static_assert(RANKS::kCount >= 1 && RANKS::kCount <= kSelNone, "at most nine targets");
  const bool tl = lane < RANKS::kCount;
  const uint32_t R = tl ? RANKS::rank(lane, N) : 0u;
  if (b >= 32) {  // a key may equal the sentinel: radix levels over every key
    uint32_t k[V];
#pragma unroll
    for (int e = 0; e < V; ++e) k[e] = keyf(e);
    return radix_select<V>(L, k, b, R, tl, lane);
  }
  // window level: bin min(key, kSelWin - 1); empty slots count in a spare word
  // of their own lane past the window (kSelWin + lane, never read), so that the
  // row's empty tail slots do not pile onto one address
  u32x4* hv = reinterpret_cast<u32x4*>(L.hist);
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[lane * 4 + i] = u32x4{0u, 0u, 0u, 0u};
  wave_lds_sync();
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const uint32_t x = keyf(e);
    if (DENSE && e % 17 != 16)
      atomicAdd(&L.hist[min(x, kSelWin - 1u)], 1u);
    else
      atomicAdd(&L.hist[x == kSelEmpty ? kSelWin + lane : min(x, kSelWin - 1u)], 1u);
    if (V > 17 && e % 17 == 16) __builtin_amdgcn_sched_barrier(0);  // bounds the addresses in flight
  }
  wave_lds_sync();
  // lane l holds bins 16 l .. 16 l + 15: their total, and the wave scan of the totals
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const u32x4 q = hv[lane * 4 + i];
    t += q.x + q.y + q.z + q.w;
  }
  const uint32_t incl = wave_incl_scan(t);
  // the lane whose bins hold each target's rank: the first whose inclusive count exceeds it
  uint32_t owner = 0;
#pragma unroll
  for (uint32_t j = 0; j < RANKS::kCount; ++j) {
    const uint32_t Rj = (uint32_t)__builtin_amdgcn_readlane((int)R, (int)j);
    const uint64_t m = ballot(incl > Rj);  // not empty: Rj < N, the total
    const uint32_t o = m ? (uint32_t)__builtin_ctzll(m) : kWave - 1u;
    if (lane == j) owner = o;
  }
  const uint32_t below = (uint32_t)__shfl((int)(incl - t), (int)owner);  // keys in the owner's lower lanes
  uint32_t key = 0, r = 0;
  bool last = false;
  if (tl) {
    r = R - below;  // rank within the owner's 16 bins
    uint32_t bin = owner * 16u;
    bool found = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const u32x4 q = hv[owner * 4 + i];
      const uint32_t c[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (!found) {
          if (r < c[e]) {
            found = true;
          } else {
            r -= c[e];
            ++bin;
          }
        }
      }
    }
    key = bin;
    last = bin == kSelWin - 1u;  // keys >= kSelWin - 1: rank r among them
  }
  wave_lds_sync();
  if (ballot(last) == 0) return key;
  // targets in the last bin: radix levels over its keys, relative to its first value
  uint32_t k[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const uint32_t x = keyf(e);
    k[e] = (x != kSelEmpty && x >= kSelWin - 1u) ? x - (kSelWin - 1u) : kSelEmpty;
  }
  const uint32_t kk = radix_select<V>(L, k, b, r, last, lane);
  return last ? kk + (kSelWin - 1u) : key;
}

// The same over a key array k[] (consumed).
template <int V, class RANKS>
__device__ __forceinline__ uint32_t wave_select(SelLds& L, uint32_t (&k)[V], uint32_t b, uint32_t N,
                                                uint32_t lane) {
  return wave_select_fn<V, RANKS, false>(L, [&](int e) { return k[e]; }, b, N, lane);
}

// Batches of one row (NB of them; batches past the row's last are empty).
template <int NB>
__device__ __forceinline__ void load_row(Batch (&B)[NB], const uint32_t* __restrict__ samples, uint64_t e0,
                                         uint32_t N, uint32_t lane) {
  const RowGeo g = row_geo(samples, e0, N);
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    if ((uint32_t)u < g.nb) {
      load_batch(B[u], samples, g, u, lane);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) B[u].q[q] = u32x4{0u, 0u, 0u, 0u};
      B[u].x = 0;
      B[u].m = 0;
    }
  }
}

// Wave totals of a 32-bit and a 64-bit per-lane sum, returned wave-uniform.
__device__ __forceinline__ void wave_total_32_64(uint32_t& a, uint64_t& c) {
  a += dpp<kDppXor1>(a);
  dpp_add64<kDppXor1>(c);
  a += dpp<kDppXor2>(a);
  dpp_add64<kDppXor2>(c);
  a += dpp<kDppHalfMirror>(a);
  dpp_add64<kDppHalfMirror>(c);
  a += dpp<kDppMirror>(a);
  dpp_add64<kDppMirror>(c);
  a += dpp<kDppBcast15, 0xA>(a);
  dpp_add64<kDppBcast15, 0xA>(c);
  a += dpp<kDppBcast31, 0xC>(a);
  dpp_add64<kDppBcast31, 0xC>(c);
  a = (uint32_t)__builtin_amdgcn_readlane((int)a, 63);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)c, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(c >> 32), 63);
  c = ((uint64_t)hi << 32) | lo;
}

// Largest row range bit length for which a lane's V keys k < 2^b have
// sum k^2 < 2^32 (and k < 2^24, the 24-bit multiplier's operand range).
template <int V>
__host__ __device__ constexpr uint32_t fast_moment_bits() {
  uint32_t b = 0;
  while (b < 24 && (uint64_t)V * (((1ull << (b + 1)) - 1) * ((1ull << (b + 1)) - 1)) < (1ull << 32)) ++b;
  return b;
}

// One row: moments (sum r, sum r^2), minimum, maximum and the order
// statistics RANKS selects (lanes 0 .. RANKS::kCount - 1).
// With the row minimum m known first, rows of a small range accumulate the
// keys k = r - m in 32 bits (sum k, sum k^2 by the 24-bit multiplier) and
// recover sum r = sum k + N m and sum r^2 = sum k^2 + 2 m sum k + N m^2 once;
// wider rows take the 96-bit accumulation of the raw samples.
// FULL: every lane's four quads of every batch hold samples (wave-uniform),
// so only the head / tail slot needs its validity checked.
template <int NB, class RANKS, bool FULL>
__device__ __forceinline__ uint32_t row_pass_impl(SelLds& L, const Batch (&B)[NB], uint32_t N, uint32_t lane,
                                                  uint64_t& s1, uint64_t& s2, uint32_t& s2h, uint32_t& row_max,
                                                  uint32_t& dec) {
  constexpr int V = 17 * NB;
  auto quad_ok = [&](int u, int q) { return FULL || ((B[u].m >> q) & 1u) != 0u; };
  uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
  for (int u = 0; u < NB; ++u) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (quad_ok(u, q)) {
        mn = min(mn, min(min(B[u].q[q].x, B[u].q[q].y), min(B[u].q[q].z, B[u].q[q].w)));
        mx = max(mx, max(max(B[u].q[q].x, B[u].q[q].y), max(B[u].q[q].z, B[u].q[q].w)));
      }
    if (B[u].m & 16u) {
      mn = min(mn, B[u].x);
      mx = max(mx, B[u].x);
    }
  }
  const uint32_t rmin = wave_min_u32(mn), rmax = wave_max_u32(mx);
  row_max = rmax;
  const uint32_t range = rmax - rmin;
  const uint32_t b = range ? 32u - __clz(range) : 0u;
  // moments first, from the raw samples, so that the keys can take the
  // samples' registers afterwards
  if (b <= fast_moment_bits<V>()) {
    uint32_t t1 = 0;
    uint32_t t2 = 0;
    auto acc = [&](bool v, uint32_t x) {
      const uint32_t z = v ? x - rmin : 0u;
      t1 += z;
      t2 += __umul24(z, z);
    };
#pragma unroll
    for (int u = 0; u < NB; ++u) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const bool v = quad_ok(u, q);
        acc(v, B[u].q[q].x);
        acc(v, B[u].q[q].y);
        acc(v, B[u].q[q].z);
        acc(v, B[u].q[q].w);
      }
      acc((B[u].m & 16u) != 0u, B[u].x);
    }
    uint64_t t2w = t2;
    wave_total_32_64(t1, t2w);
    const u128 q2 = (u128)t2w + (u128)(2ull * rmin) * t1 + (u128)((uint64_t)rmin * rmin) * N;
    s1 = (uint64_t)t1 + (uint64_t)rmin * N;
    s2 = (uint64_t)q2;
    s2h = (uint32_t)(q2 >> 64);
  } else {
    uint32_t unused = 0xffffffffu;
    s1 = 0;
    s2 = 0;
    s2h = 0;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (quad_ok(u, q)) acc_quad(B[u].q[q], unused, s1, s2, s2h);
      if (B[u].m & 16u) acc_sample(B[u].x, unused, s1, s2, s2h);
    }
    wave_total_64_96(s1, s2, s2h);
  }
  if (b == 0) {
    dec = rmin;
    return rmin;
  }
  // key of slot e: sample - row minimum (kSelEmpty for a slot without a sample)
  auto keyf = [&](int e) -> uint32_t {
    const int u = e / 17, r = e % 17;
    if (r == 16) return (B[u].m & 16u) ? B[u].x - rmin : kSelEmpty;
    const int q = r / 4, c = r % 4;
    const uint32_t x = c == 0 ? B[u].q[q].x : (c == 1 ? B[u].q[q].y : (c == 2 ? B[u].q[q].z : B[u].q[q].w));
    return quad_ok(u, q) ? x - rmin : kSelEmpty;
  };
  dec = wave_select_fn<V, RANKS, FULL>(L, keyf, b, N, lane) + rmin;
  return rmin;
}

// SPECIALISE: rows whose batches are all full take a copy of the pass with the
// quads' validity checks compiled out. It removes VALU work but costs registers:
// measured on MI355X it speeds up the statistics kernel (13.2 -> 12.2 ms on
// 8192 x 1024 x 2048) and slows the feature kernel, whose occupancy it lowers.
template <int NB, class RANKS, bool SPECIALISE = false>
__device__ __forceinline__ uint32_t row_pass(SelLds& L, const Batch (&B)[NB], uint32_t N, uint32_t lane,
                                             uint64_t& s1, uint64_t& s2, uint32_t& s2h, uint32_t& row_max,
                                             uint32_t& dec) {
  if constexpr (SPECIALISE) {
    bool full = true;
#pragma unroll
    for (int u = 0; u < NB; ++u) full = full && (B[u].m & 15u) == 15u;
    if (ballot(!full) == 0)
      return row_pass_impl<NB, RANKS, true>(L, B, N, lane, s1, s2, s2h, row_max, dec);
  }
  return row_pass_impl<NB, RANKS, false>(L, B, N, lane, s1, s2, s2h, row_max, dec);
}

// Samples per row handled by the NB-batch feature kernel: a row of N samples
// needs ceil(floor(N / 4) / 256) batches at most.
__host__ __device__ constexpr uint32_t feat_batches(uint32_t N) {
  return (N / 4 + 4u * kWave - 1) / (4u * kWave) <= 1 ? 1u : ((N / 4 + 4u * kWave - 1) / (4u * kWave) <= 2 ? 2u : 4u);
}

}  // namespace ks

// Order statistics of rows of uint32 samples, one wave per row: the row held
// in registers (1, 2 or 4 load batches per lane) or, for longer rows, streamed
// in batches; its minimum and maximum by DPP, its moments (sum r, sum r^2)
// fused with a histogram of its keys, and a multi-rank select for up to nine
// target ranks. Used by the learned path's decile features and by the per-row
// latency statistics.
#pragma once

#include "ks_scan.hpp"
#include "ks_wave.hpp"

namespace ks {

// ------------------------------------------------------------------ deciles
// Up to nine order statistics of one row, found by one wave with no block
// barrier, over the keys r - base (the row minimum, or a provisional base at
// or below it).
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
// range needs all 32 bits): an MSD radix select over the keys of that bin.
// Level 0 histograms the top kSelW0 bits of every key; each later level
// histograms the next kSelW bits (kSelWs in stream_select) of only the keys
// that share a target's prefix so far. Those keys form at most nine groups (one per distinct prefix among
// the targets), numbered in target order; histograms are LDS counters per
// (group, digit) bin. Two forms:
//   radix_select  keeps the keys in registers (the key arrays of the workflow
//                 checks) and rewrites each key after a level as
//                 (group << s) | (its s low bits), s the bits still unresolved,
//                 with group kSelNone for keys outside every group, so the next
//                 level's bin is one shift; keys past the live groups issue no
//                 LDS access (they would pile onto a few addresses);
//   stream_select reads the row again from memory at every level and finds a
//                 key's group by comparing its prefix with the groups'
//                 prefixes, so the row pass keeps no copy of the row for this
//                 rare case.

constexpr uint32_t kSelWin = 1024; // bins of the window level: keys 0 .. 1022 one each, 1023 the rest
constexpr uint32_t kSelW0 = 10;    // bits of the level-0 digit (1024 bins fit the histogram)
constexpr uint32_t kSelW = 7;      // bits of every later digit
constexpr uint32_t kSelNone = 9;   // group of keys outside every target's prefix
constexpr uint32_t kSelEmpty = 0xffffffffu;  // key of a slot without a sample

// Row classes of the row passes (feat_batches): 1, 2, 4 load batches per row
// held in registers, kStreamed rows read in batches, kGrouped short rows four
// to a wave.
constexpr uint32_t kStreamed = 8;
constexpr uint32_t kGrouped = 16;

struct __align__(16) SelLds {
  uint32_t hist[(kSelNone + 1) << kSelW];  // bin counts, then exclusive prefixes
  uint8_t tab[(kSelNone + 1) << kSelW];    // bin -> group at the next level
};

// The row pass's share of LDS per wave: the window, which stream_select's
// levels reuse (later digits of kSelWs bits, so that nine groups' bins fit),
// and the groups' prefixes. 4.2 KiB, so that eight waves per SIMD fit.
constexpr uint32_t kSelWs = 6;
struct __align__(16) RowLds {
  uint32_t hist[kSelWin];
  uint32_t gp[16];
};
static_assert((kSelNone << kSelWs) <= kSelWin && (1u << kSelW0) <= kSelWin, "stream_select's bins fit the window");
static_assert((1u << kSelW0) <= ((kSelNone + 1) << kSelW), "level-0 bins fit the histogram");
static_assert(kSelWin == 16u * kWave && kSelWin + kWave <= ((kSelNone + 1) << kSelW),
              "16 window bins per lane and a spare word per lane fit");
static_assert((((kSelNone << kSelW) + 255u) & ~255u) <= ((kSelNone + 1) << kSelW), "padded live bins fit");

// Output store of the row passes: plain for one-batch and short rows, whose outputs are
// the larger share of the traffic (the learned step on 4096 x 256 rows of 1024
// samples ran 1.6% faster than with nontemporal stores), nontemporal for longer
// rows (plain stores made the 8192 x 1024 x 2048 step 2 - 5% slower).
template <int NB, typename T>
__device__ __forceinline__ void row_out_store(T v, T* p) {
  if constexpr (NB == 1 || NB == (int)kGrouped)
    *p = v;
  else
    __builtin_nontemporal_store(v, p);
}

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

// The same with full 32-bit counts (rows of 2^16 samples or more), one
// 256-bin block per wave scan.
__device__ __forceinline__ void wave_excl_prefix32(uint32_t* hist, uint32_t nblk, uint32_t lane) {
  uint32_t base = 0;
  for (uint32_t i = 0; i < nblk; ++i) {
    u32x4* pa = reinterpret_cast<u32x4*>(hist + 256u * i + 4u * lane);
    const u32x4 a = *pa;
    const uint32_t sa = a.x + a.y + a.z + a.w;
    const uint32_t incl = wave_incl_scan(sa);
    const uint32_t ea = base + incl - sa;
    *pa = u32x4{ea, ea + a.x, ea + a.x + a.y, ea + a.x + a.y + a.z};
    base += (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
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

// Resolves the targets from a window histogram already in L.hist (bins
// 0 .. kSelWin - 2 count keys of that value, bin kSelWin - 1 every larger key;
// N keys in all). Lane j < RANKS::kCount gets the bin of the key of rank
// RANKS::rank(j, N); a target whose bin is the last one gets last = true and
// r, its rank among the keys of that bin.
template <class RANKS, class LDS>
__device__ __forceinline__ uint32_t window_find(LDS& L, uint32_t N, uint32_t lane, uint32_t& r, bool& last) {
  static_assert(RANKS::kCount >= 1 && RANKS::kCount <= kSelNone, "at most nine targets");
  const bool tl = lane < RANKS::kCount;
  wave_lds_sync();
  const u32x4* hv = reinterpret_cast<const u32x4*>(L.hist);
  // lane l holds bins 16 l .. 16 l + 15: their total, and the wave scan of the totals
  uint32_t t = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const u32x4 q = hv[lane * 4 + i];
    t += q.x + q.y + q.z + q.w;
  }
  const uint32_t incl = wave_incl_scan(t);
  // per target (its rank is wave-uniform): the first lane whose inclusive
  // count exceeds it owns the target's bin; lane j keeps target j's rank and owner
  uint32_t owner = 0, R = 0;
#pragma unroll
  for (uint32_t j = 0; j < RANKS::kCount; ++j) {
    const uint32_t Rj = RANKS::rank(j, N);
    const uint64_t m = ballot(incl > Rj);  // not empty: Rj < N, the total
    const uint32_t o = (uint32_t)__builtin_ctzll(m);
    if (lane == j) {
      owner = o;
      R = Rj;
    }
  }
  const uint32_t below = (uint32_t)__shfl((int)(incl - t), (int)owner);  // keys in the owner's lower lanes
  uint32_t key = 0;
  r = 0;
  last = false;
  if (tl) {
    // rank r within the owner's 16 bins: its bin is the number of bins whose
    // inclusive count is <= r (branch-free: one compare and two selects per bin)
    r = R - below;
    uint32_t cum = 0, nb = 0, under = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const u32x4 q = hv[owner * 4 + i];
      const uint32_t c[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cum += c[e];
        const bool le = cum <= r;
        nb += le ? 1u : 0u;
        under = le ? cum : under;
      }
    }
    key = owner * 16u + nb;
    r -= under;
    last = key == kSelWin - 1u;  // keys >= kSelWin - 1: rank r among them
  }
  wave_lds_sync();
  return key;
}

// key(e), e < V: this lane's keys (values - row minimum, empty slots
// kSelEmpty); b >= 1 the bit length of the range. Lane j < RANKS::kCount
// returns the key of rank RANKS::rank(j, N), N the number of keys in the wave
// (wave-uniform).
template <int V, class RANKS, class KeyFn>
__device__ __forceinline__ uint32_t wave_select_fn(SelLds& L, KeyFn&& keyf, uint32_t b, uint32_t N, uint32_t lane) {
  if (b >= 32) {  // a key may equal the sentinel: radix levels over every key
    const bool tl = lane < RANKS::kCount;
    const uint32_t R = tl ? RANKS::rank(lane, N) : 0u;
    uint32_t k[V];
#pragma unroll
    for (int e = 0; e < V; ++e) k[e] = keyf(e);
    return radix_select<V>(L, k, b, R, tl, lane);
  }
  // window level: bin min(key, kSelWin - 1); empty slots count in a spare word
  // of their own lane past the window (kSelWin + lane, never read), so that
  // they do not pile onto one address
  u32x4* hv = reinterpret_cast<u32x4*>(L.hist);
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[lane * 4 + i] = u32x4{0u, 0u, 0u, 0u};
  wave_lds_sync();
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const uint32_t x = keyf(e);
    atomicAdd(&L.hist[x == kSelEmpty ? kSelWin + lane : min(x, kSelWin - 1u)], 1u);
    if (V > 17 && e % 17 == 16) __builtin_amdgcn_sched_barrier(0);  // bounds the addresses in flight
  }
  uint32_t r;
  bool last;
  const uint32_t key = window_find<RANKS>(L, N, lane, r, last);
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
  return wave_select_fn<V, RANKS>(L, [&](int e) { return k[e]; }, b, N, lane);
}

// Batches of one row (NB of them; batches past the row's last are empty).
template <int NB>
__device__ __forceinline__ RowGeo load_row(Batch (&B)[NB], const uint32_t* __restrict__ samples, uint64_t e0,
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
  return g;
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

// The same for a < 2^26 and c < 2^48 per lane (the fast moments of a row
// held in registers: at most 68 keys below 2^13 per lane): c is reduced as its
// low 16 bits and the rest, whose wave totals each fit 32 bits, so every step
// is a 32-bit DPP add.
__device__ __forceinline__ void wave_total_fast_moments(uint32_t& a, uint64_t& c) {
  uint32_t lo = (uint32_t)c & 0xffffu, hi = (uint32_t)(c >> 16);
  a += dpp<kDppXor1>(a);
  lo += dpp<kDppXor1>(lo);
  hi += dpp<kDppXor1>(hi);
  a += dpp<kDppXor2>(a);
  lo += dpp<kDppXor2>(lo);
  hi += dpp<kDppXor2>(hi);
  a += dpp<kDppHalfMirror>(a);
  lo += dpp<kDppHalfMirror>(lo);
  hi += dpp<kDppHalfMirror>(hi);
  a += dpp<kDppMirror>(a);
  lo += dpp<kDppMirror>(lo);
  hi += dpp<kDppMirror>(hi);
  a += dpp<kDppBcast15, 0xA>(a);
  lo += dpp<kDppBcast15, 0xA>(lo);
  hi += dpp<kDppBcast15, 0xA>(hi);
  a += dpp<kDppBcast31, 0xC>(a);
  lo += dpp<kDppBcast31, 0xC>(lo);
  hi += dpp<kDppBcast31, 0xC>(hi);
  a = (uint32_t)__builtin_amdgcn_readlane((int)a, 63);
  lo = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
  hi = (uint32_t)__builtin_amdgcn_readlane((int)hi, 63);
  c = (uint64_t)lo + ((uint64_t)hi << 16);
}

// Largest row range bit length for which n keys k < 2^b have sum k^2 < 2^32
// (and k < 2^24, the 24-bit multiplier's operand range).
__host__ __device__ constexpr uint32_t fast_moment_bits(uint32_t n) {
  uint32_t b = 0;
  while (b < 24 && (uint64_t)n * (((1ull << (b + 1)) - 1) * ((1ull << (b + 1)) - 1)) < (1ull << 32)) ++b;
  return b;
}
constexpr uint32_t kFastBits = fast_moment_bits(17);  // per load batch (17 samples per lane)

// Calls quad(v) for every 16-byte quad of the row this lane holds and one(x)
// for its head / tail sample, then batch_end() after each batch. Batches past
// the row's last, full batches and batches without a head or tail sample are
// told apart by wave-uniform tests (g is the row's geometry), so only a
// partial batch pays a per-lane validity test.
template <int NB, class Quad, class One, class End>
__device__ __forceinline__ void for_row(const Batch (&B)[NB], const RowGeo& g, Quad&& quad, One&& one,
                                        End&& batch_end) {
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    if ((uint32_t)u >= g.nb) break;
    if ((uint32_t)(u + 1) * (4u * kWave) <= g.nq) {
#pragma unroll
      for (int q = 0; q < 4; ++q) quad(B[u].q[q]);
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((B[u].m >> q) & 1u) quad(B[u].q[q]);
    }
    if ((uint32_t)u + 1u == g.nb && (g.head | g.tail) != 0u && (B[u].m & 16u)) one(B[u].x);
    batch_end();
    __builtin_amdgcn_sched_barrier(0);  // one batch's LDS addresses in flight at a time
  }
}

// Row summary from row_scan, the input of row_select.
struct RowScan {
  uint32_t rmin, rmax;
  uint32_t b;  // bit length of rmax - rmin
};

// One row (loaded by load_row with geometry g), first part: minimum, maximum,
// moments (sum r, sum r^2) and the window histogram of the keys r - m (m the
// row minimum) in L. A first pass takes the minimum and maximum; rows of a
// range below 2^kFastBits then make one pass that sums k = r - m and k^2 in
// 32 bits per batch (24-bit multiplier) and counts each key, and recover
// sum r = sum k + N m, sum r^2 = sum k^2 + 2 m sum k + N m^2 once; wider rows
// sum the raw samples in 96 bits and count the keys in a second pass. B is
// not read after this returns, so the caller may load the next row into it
// while row_select runs.
template <int NB>
__device__ __forceinline__ RowScan row_scan(RowLds& L, const Batch (&B)[NB], const RowGeo& g, uint32_t N,
                                            uint64_t& s1, uint64_t& s2, uint32_t& s2h, uint32_t lane) {
  // clear the window now: the LDS writes overlap the minimum / maximum pass
  u32x4* hv = reinterpret_cast<u32x4*>(L.hist);
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[lane * 4 + i] = u32x4{0u, 0u, 0u, 0u};
  uint32_t mn = 0xffffffffu, mx = 0u;
  for_row(
      B, g,
      [&](const u32x4& v) {
        mn = min(mn, min(min(v.x, v.y), min(v.z, v.w)));
        mx = max(mx, max(max(v.x, v.y), max(v.z, v.w)));
      },
      [&](uint32_t x) {
        mn = min(mn, x);
        mx = max(mx, x);
      },
      [] {});
  RowScan rs;
  rs.rmin = wave_min_u32(mn);
  rs.rmax = wave_max_u32(mx);
  const uint32_t rmin = rs.rmin;
  const uint32_t range = rs.rmax - rmin;
  rs.b = range ? 32u - __clz(range) : 0u;
  uint32_t* hist = L.hist;
  wave_lds_sync();
  if (rs.b <= kFastBits) {
    uint32_t t1 = 0, t2b = 0;
    uint64_t t2 = 0;
    auto one = [&](uint32_t x) {
      const uint32_t z = x - rmin;
      t1 += z;
      t2b = __umul24(z, z) + t2b;
      atomicAdd(&hist[min(z, kSelWin - 1u)], 1u);
    };
    for_row(
        B, g,
        [&](const u32x4& v) {
          one(v.x);
          one(v.y);
          one(v.z);
          one(v.w);
        },
        one,
        [&] {
          t2 += t2b;
          t2b = 0;
        });
    wave_total_fast_moments(t1, t2);
    const u128 q2 = (u128)t2 + (u128)(2ull * rmin) * t1 + (u128)((uint64_t)rmin * rmin) * N;
    s1 = (uint64_t)t1 + (uint64_t)rmin * N;
    s2 = (uint64_t)q2;
    s2h = (uint32_t)(q2 >> 64);
  } else {
    uint32_t unused = 0xffffffffu;
    s1 = 0;
    s2 = 0;
    s2h = 0;
    for_row(
        B, g, [&](const u32x4& v) { acc_quad(v, unused, s1, s2, s2h); },
        [&](uint32_t x) { acc_sample(x, unused, s1, s2, s2h); }, [] {});
    wave_total_64_96(s1, s2, s2h);
    if (rs.b < 32) {
      auto one = [&](uint32_t x) { atomicAdd(&hist[min(x - rmin, kSelWin - 1u)], 1u); };
      for_row(
          B, g,
          [&](const u32x4& v) {
            one(v.x);
            one(v.y);
            one(v.z);
            one(v.w);
          },
          one, [] {});
    }
  }
  return rs;
}

// The same for a row whose window is based at p, a provisional base (the
// previous row's minimum less kRowMargin): one pass over the registers takes
// the minimum and maximum, sums k = r - p and k^2 in 32 bits per batch and
// counts every key, so the counting does not wait for the row's minimum. It
// holds when the row's minimum is >= p and its maximum - p < 2^kFastBits;
// false otherwise (moments and window are then not valid, the caller runs
// row_scan on the registers, which are still intact).
constexpr uint32_t kRowMargin = 128;

template <int NB>
__device__ __forceinline__ bool row_scan_based(RowLds& L, const Batch (&B)[NB], const RowGeo& g, uint32_t N,
                                               uint32_t p, uint64_t& s1, uint64_t& s2, uint32_t& s2h, RowScan& rs,
                                               uint32_t lane) {
  u32x4* hv = reinterpret_cast<u32x4*>(L.hist);
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[lane * 4 + i] = u32x4{0u, 0u, 0u, 0u};
  wave_lds_sync();
  uint32_t* hist = L.hist;
  uint32_t mn = 0xffffffffu, mx = 0u, t1 = 0, t2b = 0;
  uint64_t t2 = 0;
  auto one = [&](uint32_t x) {
    mn = min(mn, x);
    mx = max(mx, x);
    const uint32_t z = x - p;  // wraps for x < p: the row is then rejected below
    t1 += z;
    t2b = __umul24(z, z) + t2b;
    atomicAdd(&hist[min(z, kSelWin - 1u)], 1u);
  };
  for_row(
      B, g,
      [&](const u32x4& v) {
        one(v.x);
        one(v.y);
        one(v.z);
        one(v.w);
      },
      one,
      [&] {
        t2 += t2b;
        t2b = 0;
      });
  rs.rmin = wave_min_u32(mn);
  rs.rmax = wave_max_u32(mx);
  const uint32_t range = rs.rmax - rs.rmin;
  rs.b = range ? 32u - __clz(range) : 0u;
  if (rs.rmin < p || rs.rmax - p >= (1u << kFastBits)) return false;
  wave_total_fast_moments(t1, t2);
  const u128 q2 = (u128)t2 + (u128)(2ull * p) * t1 + (u128)((uint64_t)p * p) * N;
  s1 = (uint64_t)t1 + (uint64_t)p * N;
  s2 = (uint64_t)q2;
  s2h = (uint32_t)(q2 >> 64);
  return true;
}

// MSD radix levels over the keys k = r - m - off of the row's samples with
// r - m >= off (m = rmin), for targets (lanes with tl, at most kSelNone of
// them, consecutive, ranks R non-decreasing with the lane; R counts among
// those keys), every key below 2^bits. The row is read again from memory one
// batch at a time at every level, so that no copy of it stays in registers:
// this path serves only targets past the window and rows of a range of 2^31
// or more. The key's group at a level is the index of its prefix among the
// groups' prefixes (kept in LDS), compared one by one. Counts are full 32-bit
// (rows of any length).
__device__ __forceinline__ uint32_t stream_select(RowLds& L, const uint32_t* __restrict__ samples, const RowGeo& g,
                                               uint32_t rmin, uint32_t off, uint32_t bits, uint32_t R, bool tl,
                                               uint32_t lane) {
  uint32_t* gp = L.gp;  // prefixes of the groups, in target order
  const uint64_t tm = ballot(tl);
  const uint32_t first = tm ? (uint32_t)__builtin_ctzll(tm) : 0u;
  uint32_t tg = 0, key = 0, G = 1, sprev = bits, wmax = kSelW0;
  bool level0 = true;  // every key (below 2^bits) is in group 0
#pragma unroll 1
  for (;;) {
    const uint32_t w = min(sprev, wmax);
    const uint32_t s = sprev - w;
    const uint32_t nblk = ((G << w) + 255u) >> 8;
    for (uint32_t i = 0; i < nblk; ++i)
      *reinterpret_cast<u32x4*>(L.hist + 256u * i + 4u * lane) = u32x4{0u, 0u, 0u, 0u};
    wave_lds_sync();
    const uint32_t dmask = (1u << w) - 1u;
    auto count = [&](uint32_t x) {
      const uint32_t z = x - rmin;
      if (z >= off) {
        const uint32_t k = z - off;
        uint32_t gid = 0;
        if (!level0) {
          const uint32_t h = k >> sprev;
          gid = kSelNone;
          for (uint32_t q = 0; q < G; ++q)
            if (gp[q] == h) gid = q;
        }
        if (gid < G) atomicAdd(&L.hist[(gid << w) | ((k >> s) & dmask)], 1u);
      }
    };
#pragma unroll 1
    for (uint32_t u = 0; u < g.nb; ++u) {
      Batch t;
      load_batch(t, samples, g, u, lane);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((t.m >> q) & 1u) {
          count(t.q[q].x);
          count(t.q[q].y);
          count(t.q[q].z);
          count(t.q[q].w);
        }
      if (t.m & 16u) count(t.x);
    }
    wave_lds_sync();
    wave_excl_prefix32(L.hist, nblk, lane);
    wave_lds_sync();
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
    // the previous lane's bin, across DPP rows (the targets of a short row
    // grouped four to a wave may straddle lanes 15 | 16 or 31 | 32)
    const uint32_t prev = (uint32_t)__shfl((int)x, (int)(lane ? lane - 1u : 0u));
    const bool fresh = tl && (lane == first || x != prev);
    const uint64_t m = ballot(fresh);
    const uint32_t id = mbcnt(m) - (fresh ? 0u : 1u);
    wave_lds_sync();
    if (fresh) gp[id] = key;
    wave_lds_sync();
    tg = id;
    G = (uint32_t)__popcll(m);
    sprev = s;
    wmax = kSelWs;
    level0 = false;
  }
  return key;
}

// One row, second part (after row_scan): lane j < RANKS::kCount returns the
// sample of rank RANKS::rank(j, N) in the row.
template <int NB, class RANKS>
__device__ __forceinline__ uint32_t row_select(RowLds& L, const uint32_t* __restrict__ samples, const RowGeo& g,
                                               const RowScan& rs, uint32_t N, uint32_t lane) {
  if (rs.b == 0) return rs.rmin;
  uint32_t key = 0, r, off, bits;
  bool last;
  if (rs.b >= 32) {  // no window: radix levels over every key
    last = lane < RANKS::kCount;
    r = last ? RANKS::rank(lane, N) : 0u;
    off = 0;
    bits = 32;
  } else {
    key = window_find<RANKS>(L, N, lane, r, last);
    if (ballot(last) == 0) return key + rs.rmin;
    // targets in the last bin: radix levels over its keys, relative to its first value
    off = kSelWin - 1u;
    const uint32_t top = rs.rmax - rs.rmin - off;
    bits = top ? 32u - __clz(top) : 1u;
  }
  const uint32_t kk = stream_select(L, samples, g, rs.rmin, off, bits, r, last, lane);
  return (last ? kk + off : key) + rs.rmin;
}

// ------------------------------------------------------- rows of any length
// Rows longer than four load batches per lane (N > 4096 + 3) do not fit in
// registers; one wave streams them in batches of 16 bytes x 4 per lane, the
// next batch always in flight while the current one is summed.

// Calls one(x) for every sample of batch u of a row (geometry g) that this
// lane holds. A full batch and a batch without a head / tail sample are told
// apart by wave-uniform tests, so only a partial batch pays a per-lane test.
template <class One>
__device__ __forceinline__ void for_batch(const Batch& B, const RowGeo& g, uint32_t u, One&& one) {
  if ((u + 1u) * (4u * kWave) <= g.nq) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      one(B.q[q].x);
      one(B.q[q].y);
      one(B.q[q].z);
      one(B.q[q].w);
    }
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if ((B.m >> q) & 1u) {
        one(B.q[q].x);
        one(B.q[q].y);
        one(B.q[q].z);
        one(B.q[q].w);
      }
  }
  if (u + 1u == g.nb && (g.head | g.tail) != 0u && (B.m & 16u)) one(B.x);
}

// One row's results: minimum, maximum, moments (sum r; sum r^2 as 96 bits)
// and, on lane j < RANKS::kCount, the sample of rank RANKS::rank(j, N).
struct RowOut {
  uint32_t rmin, rmax;
  uint64_t s1, s2;
  uint32_t s2h;
  uint32_t sel;
};

// Lane j < RANKS::kCount: the sample of rank RANKS::rank(j, N), from the
// window histogram in L of the keys r - base (every sample >= base).
template <class RANKS>
__device__ __forceinline__ uint32_t select_from_window(RowLds& L, const uint32_t* __restrict__ samples,
                                                       const RowGeo& g, uint32_t base, uint32_t rmax, uint32_t N,
                                                       uint32_t lane) {
  uint32_t r;
  bool last;
  const uint32_t key = window_find<RANKS>(L, N, lane, r, last);
  if (ballot(last) == 0) return key + base;
  const uint32_t off = kSelWin - 1u;
  const uint32_t top = rmax - base - off;
  const uint32_t bits = top ? 32u - __clz(top) : 1u;
  const uint32_t kk = stream_select(L, samples, g, base, off, bits, r, last, lane);
  return (last ? kk + off : key) + base;
}

// The exact path for a long row the streaming pass could not finish (a
// sample below the provisional base, or a range of 2^kFastBits or more): the
// row is read again, its moments summed in 96 bits, its keys r - rmin counted
// into a fresh window (unless the range needs all 32 bits), and the order
// statistics selected.
template <class RANKS>
__device__ __forceinline__ void row_exact(RowLds& L, const uint32_t* __restrict__ samples, const RowGeo& g,
                                          uint32_t N, uint32_t lane, RowOut& o) {
  const uint32_t rmin = o.rmin;
  const uint32_t range = o.rmax - rmin;
  const uint32_t b = range ? 32u - __clz(range) : 0u;
  u32x4* hv = reinterpret_cast<u32x4*>(L.hist);
#pragma unroll
  for (int i = 0; i < 4; ++i) hv[lane * 4 + i] = u32x4{0u, 0u, 0u, 0u};
  wave_lds_sync();
  uint32_t unused = 0xffffffffu;
  uint64_t s1 = 0, s2 = 0;
  uint32_t s2h = 0;
  const bool window = b >= 1 && b < 32;
#pragma unroll 1
  for (uint32_t u = 0; u < g.nb; ++u) {
    Batch t;
    load_batch(t, samples, g, u, lane);
    for_batch(t, g, u, [&](uint32_t x) {
      acc_sample(x, unused, s1, s2, s2h);
      if (window) atomicAdd(&L.hist[min(x - rmin, kSelWin - 1u)], 1u);
    });
  }
  wave_total_64_96(s1, s2, s2h);
  o.s1 = s1;
  o.s2 = s2;
  o.s2h = s2h;
  if (b == 0) {
    o.sel = rmin;
  } else if (window) {
    o.sel = select_from_window<RANKS>(L, samples, g, rmin, o.rmax, N, lane);
  } else {  // no window: radix levels over every key
    const bool tl = lane < RANKS::kCount;
    const uint32_t R = tl ? RANKS::rank(lane, N) : 0u;
    o.sel = stream_select(L, samples, g, rmin, 0u, 32u, R, tl, lane) + rmin;
  }
}

// Rows first, first + step, ... (below K) of a [K][N] block at element off0,
// streamed by one wave; emit(i, o) receives each row's results. The two batch
// buffers alternate, so no copy moves between them.
//
// Per row: the first batch's minimum m0, less a margin kSelMargin, is the
// provisional base a; every sample then adds k = r - a to sums of k and k^2
// (32-bit within a batch, 64-bit across batches; 24-bit multiplier) and
// counts bin min(k, kSelWin - 1) of the window histogram. With the row's true
// minimum m and maximum M at its end: if m >= a and M - a < 2^kFastBits, the
// sums give sum r = sum k + N a and sum r^2 = sum k^2 + 2 a sum k + N a^2
// exactly and the histogram (based at a) gives the order statistics;
// otherwise row_exact reads the row again.
constexpr uint32_t kSelMargin = 128;

template <class RANKS, class Emit>
__device__ __forceinline__ void select_rows_long(RowLds& L, const uint32_t* __restrict__ samples, uint64_t off0,
                                                 uint32_t N, uint32_t K, uint32_t first, uint32_t step, uint32_t lane,
                                                 Emit&& emit) {
  struct Cursor {
    uint32_t i, u;
    RowGeo g;
  };
  auto geo = [&](uint32_t i) { return row_geo(samples, off0 + (uint64_t)i * N, N); };
  auto advance = [&](const Cursor& c) {
    Cursor n = c;
    if (c.u + 1u < c.g.nb) {
      n.u = c.u + 1u;
    } else {
      n.i = c.i + step;
      n.u = 0;
      if (n.i < K) n.g = geo(n.i);
    }
    return n;
  };
  // the row in progress
  uint32_t base = 0, mn = 0, mx = 0;
  uint64_t t1 = 0, t2 = 0;
  uint32_t* hist = L.hist;
  auto process = [&](const Batch& B, const Cursor& c) {
    if (c.u == 0) {
      // a new row: clear the window and take the provisional base from this batch
      u32x4* hv = reinterpret_cast<u32x4*>(hist);
#pragma unroll
      for (int i = 0; i < 4; ++i) hv[lane * 4 + i] = u32x4{0u, 0u, 0u, 0u};
      mn = 0xffffffffu;
      mx = 0u;
      for_batch(B, c.g, 0u, [&](uint32_t x) {
        mn = min(mn, x);
        mx = max(mx, x);
      });
      const uint32_t m0 = wave_min_u32(mn);
      base = m0 > kSelMargin ? m0 - kSelMargin : 0u;
      t1 = 0;
      t2 = 0;
      wave_lds_sync();
    }
    uint32_t t1b = 0, t2b = 0;
    auto one = [&](uint32_t x) {
      const uint32_t z = x - base;
      t1b += z;
      t2b = __umul24(z, z) + t2b;
      atomicAdd(&hist[min(z, kSelWin - 1u)], 1u);
    };
    if (c.u == 0) {
      for_batch(B, c.g, 0u, one);
    } else {
      for_batch(B, c.g, c.u, [&](uint32_t x) {
        mn = min(mn, x);
        mx = max(mx, x);
        one(x);
      });
    }
    t1 += t1b;
    t2 += t2b;
    if (c.u + 1u == c.g.nb) {  // the row's last batch
      RowOut o;
      o.rmin = wave_min_u32(mn);
      o.rmax = wave_max_u32(mx);
      if (o.rmin >= base && o.rmax - base < (1u << kFastBits)) {
        uint64_t a1 = t1, a2 = t2;
        uint32_t a2h = 0;
        wave_total_64_96(a1, a2, a2h);
        const u128 q2 = (((u128)a2h << 64) | a2) + (u128)(2ull * base) * a1 + (u128)((uint64_t)base * base) * N;
        o.s1 = a1 + (uint64_t)base * N;
        o.s2 = (uint64_t)q2;
        o.s2h = (uint32_t)(q2 >> 64);
        o.sel = o.rmax == o.rmin ? o.rmin : select_from_window<RANKS>(L, samples, c.g, base, o.rmax, N, lane);
      } else {
        row_exact<RANKS>(L, samples, c.g, N, lane, o);
      }
      emit(c.i, o);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  Cursor c;
  c.i = first;
  c.u = 0;
  if (c.i >= K) return;
  c.g = geo(c.i);
  Batch A, B;
  load_batch(A, samples, c.g, 0u, lane);
  for (;;) {
    Cursor n = advance(c);
    if (n.i < K) load_batch(B, samples, n.g, n.u, lane);
    process(A, c);
    if (n.i >= K) break;
    c = advance(n);
    if (c.i < K) load_batch(A, samples, c.g, c.u, lane);
    process(B, n);
    if (c.i >= K) break;
  }
}

// ------------------------------------------------- short rows, four to a wave
// Rows of up to kGroupMaxN samples go four to a wave, one to each 16-lane DPP
// row (g = lane / 16), loaded like the scan's grouped rows (load_group: up to
// four quads and one head or tail sample per lane). Their minimum, maximum and
// moments take four in-row DPP steps, and the four rows share one window: row
// g counts its keys in byte g of each bin (a row has at most 255 keys, so no
// byte carries into the next), so one lane-total pass, one wave scan and one
// pass over the owners' bins serve all four. Row g's targets sit on lanes
// g C .. g C + C - 1 (C = RANKS::kCount); a row whose range needs all 32 bits,
// or a row with a target past the window, takes stream_select on its own.
constexpr uint32_t kGroupMaxN = 255;
constexpr int kGroupGL = 16;
constexpr uint32_t kGroupRows = kWave / kGroupGL;

__device__ __forceinline__ uint32_t group16_min(uint32_t v) {
  v = min(v, dpp<kDppXor1>(v));
  v = min(v, dpp<kDppXor2>(v));
  v = min(v, dpp<kDppHalfMirror>(v));
  return min(v, dpp<kDppMirror>(v));
}
__device__ __forceinline__ uint32_t group16_max(uint32_t v) {
  v = max(v, dpp<kDppXor1>(v));
  v = max(v, dpp<kDppXor2>(v));
  v = max(v, dpp<kDppHalfMirror>(v));
  return max(v, dpp<kDppMirror>(v));
}
__device__ __forceinline__ uint32_t group16_sum(uint32_t v) {
  v += dpp<kDppXor1>(v);
  v += dpp<kDppXor2>(v);
  v += dpp<kDppHalfMirror>(v);
  return v + dpp<kDppMirror>(v);
}

// Rows begin .. end - 1 of one series (rows of N <= kGroupMaxN samples from
// element off0), four per step; emit(i, o, first) gets row i's results with
// its targets on lanes first .. first + C - 1 of o.sel.
template <class RANKS, class Emit>
__device__ __forceinline__ void select_rows_grouped(RowLds& L, const uint32_t* __restrict__ samples, uint64_t off0,
                                                    uint32_t N, uint32_t begin, uint32_t end, uint32_t lane,
                                                    Emit&& emit) {
  constexpr uint32_t C = RANKS::kCount;
  constexpr int GL = kGroupGL;
  static_assert(kGroupRows * C <= (uint32_t)kWave, "every row's targets have lanes");
  if (begin >= end) return;
  const uint32_t g = lane / GL, gl = lane % GL;
  const uint32_t nqu = min(4u, ((N >> 2) + GL - 1) / GL);
  const bool tl = lane < kGroupRows * C;         // a target lane: row tg, rank j
  const uint32_t tg = tl ? lane / C : 0u;
  const uint32_t R = tl ? RANKS::rank(lane % C, N) : 0u;
  uint32_t* hist = L.hist;
  u32x4* hv = reinterpret_cast<u32x4*>(hist);
  Batch cur;
  load_group<GL>(cur, samples, off0 + (uint64_t)(begin + g) * N, N, begin + g < end, gl, nqu);
  for (uint32_t i = begin; i < end; i += kGroupRows) {
    const uint32_t nrows = min(kGroupRows, end - i);
#pragma unroll
    for (int q = 0; q < 4; ++q) hv[lane * 4 + q] = u32x4{0u, 0u, 0u, 0u};
    uint32_t mn = 0xffffffffu, mx = 0u;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if ((cur.m >> u) & 1u) {
        const u32x4 v = cur.q[u];
        mn = min(mn, min(min(v.x, v.y), min(v.z, v.w)));
        mx = max(mx, max(max(v.x, v.y), max(v.z, v.w)));
      }
    if (cur.m & 16u) {
      mn = min(mn, cur.x);
      mx = max(mx, cur.x);
    }
    const uint32_t rmin = group16_min(mn), rmax = group16_max(mx);
    const bool has = g < nrows;  // every row of the step has N >= 1 samples
    const uint32_t range = has ? rmax - rmin : 0u;
    const uint32_t b = range ? 32u - __clz(range) : 0u;
    const uint32_t inc = 1u << (8u * g);
    const bool wide = ballot(has && b > kFastBits) != 0;
    uint64_t s1 = 0, s2 = 0;
    uint32_t s2h = 0;
    wave_lds_sync();  // the window is clear before any count
    if (!wide) {
      // keys z = r - rmin below 2^13: per lane at most 17 of them (t2 < 2^31),
      // per row sum z < 2^21 and sum z^2 < 2^34, the latter summed as its low
      // 16 bits and the rest
      uint32_t t1 = 0, t2 = 0;
      auto one = [&](uint32_t x) {
        const uint32_t z = x - rmin;
        t1 += z;
        t2 = __umul24(z, z) + t2;
        atomicAdd(&hist[min(z, kSelWin - 1u)], inc);
      };
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((cur.m >> u) & 1u) {
          one(cur.q[u].x);
          one(cur.q[u].y);
          one(cur.q[u].z);
          one(cur.q[u].w);
        }
      if (cur.m & 16u) one(cur.x);
      const uint32_t a = group16_sum(t1), lo = group16_sum(t2 & 0xffffu), hi = group16_sum(t2 >> 16);
      const uint64_t T2 = (uint64_t)lo + ((uint64_t)hi << 16);
      const u128 q2 = (u128)T2 + (u128)(2ull * rmin) * a + (u128)((uint64_t)rmin * rmin) * N;
      s1 = (uint64_t)a + (uint64_t)rmin * N;
      s2 = (uint64_t)q2;
      s2h = (uint32_t)(q2 >> 64);
    } else {
      uint32_t unused = 0xffffffffu;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if ((cur.m >> u) & 1u) acc_quad(cur.q[u], unused, s1, s2, s2h);
      if (cur.m & 16u) acc_sample(cur.x, unused, s1, s2, s2h);
      group_total_64_96<GL>(s1, s2, s2h);
      if (b < 32) {
        auto one = [&](uint32_t x) { atomicAdd(&hist[min(x - rmin, kSelWin - 1u)], inc); };
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if ((cur.m >> u) & 1u) {
            one(cur.q[u].x);
            one(cur.q[u].y);
            one(cur.q[u].z);
            one(cur.q[u].w);
          }
        if (cur.m & 16u) one(cur.x);
      }
    }
    // the next step's rows are in flight while this step's order statistics are found
    const uint32_t nx = i + kGroupRows;
    if (nx < end) load_group<GL>(cur, samples, off0 + (uint64_t)(nx + g) * N, N, nx + g < end, gl, nqu);
    // the window of the four rows: lane totals, wave scan, each target's owner lane
    wave_lds_sync();
    uint32_t t = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const u32x4 v = hv[lane * 4 + q];
      t += v.x + v.y + v.z + v.w;
    }
    const uint32_t incl = wave_incl_scan(t);
    uint32_t owner = 0;
#pragma unroll
    for (uint32_t rg = 0; rg < kGroupRows; ++rg) {
      const uint32_t f = (incl >> (8u * rg)) & 0xffu;
#pragma unroll
      for (uint32_t j = 0; j < C; ++j) {
        const uint64_t m = ballot(f > RANKS::rank(j, N));  // empty for a row without a window
        const uint32_t o = m ? (uint32_t)__builtin_ctzll(m) : 0u;
        if (lane == rg * C + j) owner = o;
      }
    }
    const uint32_t sh = 8u * tg;
    const uint32_t below = ((uint32_t)__shfl((int)(incl - t), (int)owner) >> sh) & 0xffu;
    uint32_t key = 0, r = 0;
    bool last = false;
    if (tl) {
      r = R - below;
      uint32_t cum = 0, nb = 0, under = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const u32x4 v = hv[owner * 4 + q];
        const uint32_t c[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cum += (c[e] >> sh) & 0xffu;
          const bool le = cum <= r;
          nb += le ? 1u : 0u;
          under = le ? cum : under;
        }
      }
      key = owner * 16u + nb;
      r -= under;
      last = key == kSelWin - 1u;
    }
    wave_lds_sync();
    // each row's results; radix levels for a row without a window or with a
    // target past it (both rare for latency rows)
    for (uint32_t rg = 0; rg < nrows; ++rg) {
      const int src = (int)(rg * GL);
      RowOut o;
      o.rmin = (uint32_t)__builtin_amdgcn_readlane((int)rmin, src);
      o.rmax = (uint32_t)__builtin_amdgcn_readlane((int)rmax, src);
      o.s1 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(s1 >> 32), src) << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s1, src);
      o.s2 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(s2 >> 32), src) << 32) |
             (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)s2, src);
      o.s2h = (uint32_t)__builtin_amdgcn_readlane((int)s2h, src);
      const uint32_t bb = (uint32_t)__builtin_amdgcn_readlane((int)b, src);
      const bool mine = tl && tg == rg;
      o.sel = key + o.rmin;
      if (bb >= 32) {
        const RowGeo gr = row_geo(samples, off0 + (uint64_t)(i + rg) * N, N);
        const uint32_t kk = stream_select(L, samples, gr, o.rmin, 0u, 32u, R, mine, lane);
        if (mine) o.sel = kk + o.rmin;
      } else if (ballot(mine && last) != 0) {
        const RowGeo gr = row_geo(samples, off0 + (uint64_t)(i + rg) * N, N);
        const uint32_t offk = kSelWin - 1u;
        const uint32_t top = o.rmax - o.rmin - offk;
        const uint32_t bits = top ? 32u - __clz(top) : 1u;
        const uint32_t kk = stream_select(L, samples, gr, o.rmin, offk, bits, r, mine && last, lane);
        if (mine && last) o.sel = kk + offk + o.rmin;
      }
      emit(i + rg, o, rg * C);
    }
  }
}

// Row class of the order-statistics kernels: rows of up to kGroupMaxN samples
// go four to a wave (class kGrouped); otherwise a row of N samples needs
// ceil(floor(N / 4) / 256) load batches at most, and rows of up to 1, 2 or 4
// of them are held in registers (class 1, 2, 4), longer rows are streamed
// (class kStreamed).
// Waves per SIMD the row-pass kernels are compiled for, by row class (1 = the
// compiler's choice). With 4.3 KiB of LDS per wave the register file sets the
// occupancy; these are the largest targets met without spills (6 at 80
// registers), which run rows of up to 1027 samples 6 - 9% faster than the 5
// waves the compiler picks by itself. Rows of 2048 samples keep the
// compiler's 4 (5 spills and runs slower), and so do short rows (higher
// targets spill).
__host__ __device__ constexpr int feat_waves_per_eu(int NB) { return NB == 1 ? 6 : NB == 4 ? 3 : 1; }
__host__ __device__ constexpr int stats_waves_per_eu(int NB) { return NB == 1 ? 6 : 1; }
// Workgroup threads of the row-pass kernels by row class: rows of two load
// batches (1028 - 2051 samples) run in 512-thread workgroups, eight waves on
// a series (two workgroups per CU at the same four waves per SIMD; 1% faster
// than 256 threads on 8192 x 1024 x 2048), the other classes in 256.
__host__ __device__ constexpr int row_pass_threads(int NB) { return NB == 2 ? 512 : 256; }
__host__ __device__ constexpr uint32_t feat_batches(uint32_t N) {
  return N <= kGroupMaxN ? kGrouped
         : (N / 4 + 4u * kWave - 1) / (4u * kWave) <= 1
             ? 1u
             : ((N / 4 + 4u * kWave - 1) / (4u * kWave) <= 2
                    ? 2u
                    : ((N / 4 + 4u * kWave - 1) / (4u * kWave) <= 4 ? 4u : kStreamed));
}

}  // namespace ks

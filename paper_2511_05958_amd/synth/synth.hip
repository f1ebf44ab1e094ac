// Seeded synthetic latency-versus-footprint sweeps.
//
// This is an input generator only: it holds none of the change-point method's
// arithmetic. It draws series shaped like the 2-D timing array of the size
// benchmarks (one row per array size, the first N load latencies of that size,
// Section "Size benchmarks", workflow steps 2 and 4) with planted latency
// plateaus, ramps, lognormal jitter, Pareto tails and outliers.
//
// Randomness: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11), keyed by (seed, series id); a sample's
// counter is (column j, row i, 0, 0), a series-parameter draw's counter is
// (draw index, 0, 0, 1). Every floating-point step below is an IEEE add,
// subtract, multiply, divide, square root or floor, compiled without FMA
// contraction, so the host and device builds of the same function produce
// identical bits. exp, log and cos are evaluated with this file's own range
// reduction plus Taylor / atanh series instead of libm / ocml for that reason.

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <thread>
#include <vector>

#define SYN_HD __host__ __device__ __forceinline__

extern "C" {

// One synthetic series. Layout is shared with the Python wrapper (240 bytes).
typedef struct syn_series {
  uint64_t offset;         // first sample, in uint32 elements; multiple of 64 (256-byte aligned)
  uint32_t K, N;           // rows (footprint steps) and samples per row
  uint32_t sid, nseg;      // series id (Philox key word 1); number of level segments
  uint32_t nplant, pad;    // number of planted transitions; unused
  uint32_t seg_start[16];  // segment s covers rows [seg_start[s], seg_start[s+1])
  uint32_t plant[4];       // first row of each planted transition
  double seg_level[16];    // nominal latency (cycles) of each segment
} syn_series;

// Per-batch noise model.
typedef struct syn_noise {
  double sigma;         // lognormal jitter: multiplier exp(sigma * z), z ~ N(0,1)
  double p_out;         // probability that a sample is an outlier
  double out_lo, out_hi;// outlier multiplier ~ U[out_lo, out_hi]
  double p_pareto;      // probability of a Pareto(x_m = 1, alpha) multiplier instead of jitter
  double pareto_alpha;
} syn_noise;

}  // extern "C"

static_assert(sizeof(syn_series) == 240, "syn_series layout");
static_assert(sizeof(syn_noise) == 48, "syn_noise layout");

namespace {

struct u4 {
  uint32_t x, y, z, w;
};

SYN_HD u4 philox4x32_10(u4 c, uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = u4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// Uniform on (0, 1): (w + 1/2) / 2^32, exact in double.
SYN_HD double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

SYN_HD double bits_to_f64(uint64_t b) { return __builtin_bit_cast(double, b); }
SYN_HD uint64_t f64_to_bits(double d) { return __builtin_bit_cast(uint64_t, d); }

SYN_HD double syn_floor(double x) { return __builtin_floor(x); }

// exp(x) for |x| < 700: x = k ln2 + r (Cody-Waite split of ln2), |r| <= ln2/2,
// exp(r) by its Taylor polynomial to degree 13, then scaled by 2^k.
SYN_HD double syn_exp(double x) {
  const double inv_ln2 = 1.4426950408889634;
  const double ln2_hi = 6.93147180369123816490e-01;
  const double ln2_lo = 1.90821492927058770002e-10;
  const double kd = syn_floor(x * inv_ln2 + 0.5);
  const double r = (x - kd * ln2_hi) - kd * ln2_lo;
  double p = 1.6059043836821613e-10;
  p = p * r + 2.08767569878681e-09;
  p = p * r + 2.505210838544172e-08;
  p = p * r + 2.755731922398589e-07;
  p = p * r + 2.7557319223985893e-06;
  p = p * r + 2.48015873015873e-05;
  p = p * r + 0.0001984126984126984;
  p = p * r + 0.001388888888888889;
  p = p * r + 0.008333333333333333;
  p = p * r + 0.041666666666666664;
  p = p * r + 0.16666666666666666;
  p = p * r + 0.5;
  p = p * r + 1.0;
  p = p * r + 1.0;
  const int64_t k = (int64_t)kd;
  return p * bits_to_f64((uint64_t)(k + 1023) << 52);
}

// log(x) for positive normal x: x = 2^e m with m in [1/sqrt2, sqrt2),
// log m = 2 atanh(s), s = (m-1)/(m+1), by the odd series to s^25.
SYN_HD double syn_log(double x) {
  const double ln2_hi = 6.93147180369123816490e-01;
  const double ln2_lo = 1.90821492927058770002e-10;
  const uint64_t b = f64_to_bits(x);
  int e = (int)((b >> 52) & 0x7ff) - 1023;
  double m = bits_to_f64((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull);
  if (m > 1.4142135623730951) {
    m = m * 0.5;
    e += 1;
  }
  const double s = (m - 1.0) / (m + 1.0);
  const double s2 = s * s;
  double p = 0.04;
  p = p * s2 + 0.043478260869565216;
  p = p * s2 + 0.047619047619047616;
  p = p * s2 + 0.05263157894736842;
  p = p * s2 + 0.058823529411764705;
  p = p * s2 + 0.06666666666666667;
  p = p * s2 + 0.07692307692307693;
  p = p * s2 + 0.09090909090909091;
  p = p * s2 + 0.1111111111111111;
  p = p * s2 + 0.14285714285714285;
  p = p * s2 + 0.2;
  p = p * s2 + 0.3333333333333333;
  p = p * s2 + 1.0;
  const double ed = (double)e;
  return ed * ln2_hi + (ed * ln2_lo + 2.0 * s * p);
}

// cos(2 pi u) for u in [0, 1): quadrant from floor(4u), then Taylor series of
// sin / cos of the remaining angle in [0, pi/2).
SYN_HD double syn_cos2pi(double u) {
  const double v = 4.0 * u;
  const double q = syn_floor(v);
  const double a = (v - q) * 1.5707963267948966;
  const double a2 = a * a;
  double c = -8.896791392450574e-22;
  c = c * a2 + 4.110317623312165e-19;
  c = c * a2 + -1.5619206968586225e-16;
  c = c * a2 + 4.779477332387385e-14;
  c = c * a2 + -1.1470745597729725e-11;
  c = c * a2 + 2.08767569878681e-09;
  c = c * a2 + -2.755731922398589e-07;
  c = c * a2 + 2.48015873015873e-05;
  c = c * a2 + -0.001388888888888889;
  c = c * a2 + 0.041666666666666664;
  c = c * a2 + -0.5;
  c = c * a2 + 1.0;
  double s = -3.868170170630684e-23;
  s = s * a2 + 1.9572941063391263e-20;
  s = s * a2 + -8.22063524662433e-18;
  s = s * a2 + 2.8114572543455206e-15;
  s = s * a2 + -7.647163731819816e-13;
  s = s * a2 + 1.6059043836821613e-10;
  s = s * a2 + -2.505210838544172e-08;
  s = s * a2 + 2.7557319223985893e-06;
  s = s * a2 + -0.0001984126984126984;
  s = s * a2 + 0.008333333333333333;
  s = s * a2 + -0.16666666666666666;
  s = s * a2 + 1.0;
  s = s * a;
  switch ((int)q & 3) {
    case 0: return c;
    case 1: return -s;
    case 2: return -c;
    default: return s;
  }
}

// Round half up and clamp to the uint32 latency range [1, 2^32-1].
SYN_HD uint32_t round_clamp(double x) {
  const double y = syn_floor(x + 0.5);
  if (!(y >= 1.0)) return 1u;
  if (y >= 4294967295.0) return 0xffffffffu;
  return (uint32_t)y;
}

SYN_HD double level_at(const syn_series& s, uint32_t i) {
  double L = s.seg_level[0];
  for (uint32_t t = 1; t < s.nseg; ++t)
    if (i >= s.seg_start[t]) L = s.seg_level[t];
  return L;
}

SYN_HD uint32_t sample_at(const syn_series& s, const syn_noise& nz, uint32_t seed,
                          double L, uint32_t i, uint32_t j) {
  const u4 w = philox4x32_10(u4{j, i, 0u, 0u}, seed, s.sid);
  const double u0 = u01(w.x);
  double x;
  if (u0 < nz.p_out) {
    x = L * (nz.out_lo + (nz.out_hi - nz.out_lo) * u01(w.w));
  } else if (u0 < nz.p_out + nz.p_pareto) {
    x = L * syn_exp(-syn_log(u01(w.w)) / nz.pareto_alpha);
  } else {
    const double z = __builtin_sqrt(-2.0 * syn_log(u01(w.y))) * syn_cos2pi(u01(w.z));
    x = L * syn_exp(nz.sigma * z);
  }
  return round_clamp(x);
}

// ---- series-parameter draws (host) ----

struct Draw {
  uint32_t seed, sid, n = 0;
  uint32_t next() { return philox4x32_10(u4{n++, 0u, 0u, 1u}, seed, sid).x; }
  double uni() { return u01(next()); }
  uint32_t below(uint32_t m) { return (uint32_t)syn_floor(uni() * (double)m); }  // U{0..m-1}
};

void sort_u32(uint32_t* a, int n) {
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && a[j - 1] > a[j]; --j) {
      uint32_t t = a[j];
      a[j] = a[j - 1];
      a[j - 1] = t;
    }
}

// Random ascending subset of size k from ladder[0..n).
void pick_levels(Draw& d, const double* ladder, int n, int k, double spread, double* out) {
  uint32_t idx[8];
  for (int i = 0; i < n; ++i) idx[i] = (uint32_t)i;
  for (int i = 0; i < k; ++i) {
    const uint32_t j = (uint32_t)i + d.below((uint32_t)(n - i));
    const uint32_t t = idx[i];
    idx[i] = idx[j];
    idx[j] = t;
  }
  sort_u32(idx, k);
  for (int i = 0; i < k; ++i) out[i] = ladder[idx[i]] * (1.0 - spread + 2.0 * spread * d.uni());
}

// Plateau lengths >= minlen summing to total: the slack is cut at nlev-1 sorted uniform points.
void plateau_lengths(Draw& d, int nlev, uint32_t total, uint32_t minlen, uint32_t* len) {
  const uint32_t slack = total - minlen * (uint32_t)nlev;
  uint32_t cut[8];
  for (int t = 0; t < nlev - 1; ++t) cut[t] = d.below(slack + 1);
  sort_u32(cut, nlev - 1);
  uint32_t prev = 0;
  for (int t = 0; t < nlev; ++t) {
    const uint32_t c = (t < nlev - 1) ? cut[t] : slack;
    len[t] = minlen + (c - prev);
    prev = c;
  }
}

// Lay out plateaus (and optional 2-row ramps at 1/3 and 2/3 of each jump).
void layout(syn_series* s, int nlev, const double* lev, const uint32_t* len, bool ramps) {
  uint32_t row = 0;
  int ns = 0;
  s->nplant = 0;
  for (int t = 0; t < nlev; ++t) {
    if (t > 0) {
      s->plant[s->nplant++] = row;
      if (ramps) {
        const double jump = lev[t] - lev[t - 1];
        s->seg_start[ns] = row;
        s->seg_level[ns++] = lev[t - 1] + jump / 3.0;
        s->seg_start[ns] = row + 1;
        s->seg_level[ns++] = lev[t - 1] + 2.0 * jump / 3.0;
        row += 2;
      }
    }
    s->seg_start[ns] = row;
    s->seg_level[ns++] = lev[t];
    row += len[t];
  }
  s->nseg = (uint32_t)ns;
}

int make_series(int config, uint32_t seed, uint32_t sid, syn_series* s) {
  memset(s, 0, sizeof(*s));
  s->sid = sid;
  Draw d{seed, sid};
  double lev[8];
  uint32_t len[8];
  switch (config) {
    case 1: {  // K=64, N=256, one change 120 -> 320 at a uniform row 1..63
      s->K = 64;
      s->N = 256;
      const uint32_t c0 = 1 + d.below(63);
      lev[0] = 120.0;
      lev[1] = 320.0;
      len[0] = c0;
      len[1] = 64 - c0;
      layout(s, 2, lev, len, false);
      return 0;
    }
    case 2:
    case 4: {  // K=256, N=1024, 1-4 plateaus from the 120/300/550/850 ladder +-10%, >= 8 rows each
      static const double ladder[4] = {120.0, 300.0, 550.0, 850.0};
      s->K = 256;
      s->N = 1024;
      const int nlev = 1 + (int)d.below(4);
      pick_levels(d, ladder, 4, nlev, 0.1, lev);
      plateau_lengths(d, nlev, 256, 8, len);
      layout(s, nlev, lev, len, false);
      return 0;
    }
    case 3: {  // log-uniform K in [32,512], N in [64,4096]; 0-4 ramped transitions; plateaus >= 4 rows
      static const double ladder[5] = {120.0, 300.0, 550.0, 850.0, 1300.0};
      const double ln32 = 3.4657359027997265, ln512 = 6.238324625039508;
      const double ln64 = 4.1588830833596715, ln4096 = 8.317766166719343;
      s->K = (uint32_t)syn_floor(syn_exp(ln32 + (ln512 - ln32) * d.uni()) + 0.5);
      s->N = (uint32_t)syn_floor(syn_exp(ln64 + (ln4096 - ln64) * d.uni()) + 0.5);
      int T = (int)d.below(5);
      while (T > 0 && 4u * (uint32_t)(T + 1) + 2u * (uint32_t)T > s->K) --T;
      const int nlev = T + 1;
      pick_levels(d, ladder, 5, nlev, 0.1, lev);
      plateau_lengths(d, nlev, s->K - 2u * (uint32_t)T, 4, len);
      layout(s, nlev, lev, len, true);
      return 0;
    }
    case 5: {  // K=1024, N=2048, 1-4 transitions with adjacent ratios U[1.05,1.2]
      s->K = 1024;
      s->N = 2048;
      const int nlev = 2 + (int)d.below(4);
      lev[0] = 120.0 * (0.9 + 0.2 * d.uni());
      for (int t = 1; t < nlev; ++t) lev[t] = lev[t - 1] * (1.05 + 0.15 * d.uni());
      plateau_lengths(d, nlev, 1024, 8, len);
      layout(s, nlev, lev, len, false);
      return 0;
    }
    default:
      return -1;
  }
}

__global__ __launch_bounds__(256) void fill_kernel(const syn_series* __restrict__ specs,
                                                   syn_noise nz, uint32_t seed,
                                                   uint32_t* __restrict__ dst, uint64_t base) {
  const syn_series& s = specs[blockIdx.y];
  const uint32_t total = s.K * s.N;
  uint32_t* out = dst + (s.offset - base);
  for (uint32_t idx = blockIdx.x * 256u + threadIdx.x; idx < total; idx += gridDim.x * 256u) {
    const uint32_t i = idx / s.N, j = idx - i * s.N;
    out[idx] = sample_at(s, nz, seed, level_at(s, i), i, j);
  }
}

}  // namespace

extern "C" {

// Noise model of each workload recipe.
int syn_noise_for(int config, syn_noise* nz) {
  if (!nz) return -1;
  *nz = syn_noise{0.08, 0.01, 1.0, 5.0, 0.0, 2.5};
  switch (config) {
    case 1: nz->sigma = 0.05; nz->p_out = 0.0; return 0;
    case 2: case 3: case 4: return 0;
    case 5: nz->p_out = 0.05; nz->p_pareto = 0.10; return 0;
    default: return -1;
  }
}

// Series specs for ids first_sid .. first_sid+num-1, packed back to back with
// 256-byte aligned bases starting at element 0. Returns the buffer length in
// elements through total_elems.
int syn_make_batch(int config, uint32_t seed, uint32_t first_sid, uint32_t num,
                   syn_series* out, uint64_t* total_elems) {
  if ((!out && num) || !total_elems) return -1;
  uint64_t off = 0;
  for (uint32_t t = 0; t < num; ++t) {
    if (make_series(config, seed, first_sid + t, &out[t])) return -1;
    out[t].offset = off;
    off += ((uint64_t)out[t].K * out[t].N + 63) & ~(uint64_t)63;
  }
  *total_elems = off;
  return 0;
}

// Fill series into a host buffer; series t lands at dst[specs[t].offset - base].
int syn_fill_host(const syn_series* specs, uint32_t num, const syn_noise* nz, uint32_t seed,
                  uint32_t* dst, uint64_t base, uint64_t dst_elems, int threads) {
  if ((!specs || !dst) && num) return -1;
  if (!nz) return -1;
  for (uint32_t t = 0; t < num; ++t)
    if (specs[t].offset < base || specs[t].offset - base + (uint64_t)specs[t].K * specs[t].N > dst_elems)
      return -2;
  if (threads < 1) threads = 1;
  auto work = [&](int tid) {
    for (uint32_t t = (uint32_t)tid; t < num; t += (uint32_t)threads) {
      const syn_series& s = specs[t];
      uint32_t* o = dst + (s.offset - base);
      for (uint32_t i = 0; i < s.K; ++i) {
        const double L = level_at(s, i);
        for (uint32_t j = 0; j < s.N; ++j) o[(uint64_t)i * s.N + j] = sample_at(s, *nz, seed, L, i, j);
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& th : pool) th.join();
  return 0;
}

// Fill series into a device buffer (same bits as syn_fill_host); synchronous.
int syn_fill_device(const syn_series* specs, uint32_t num, const syn_noise* nz, uint32_t seed,
                    uint32_t* dst, uint64_t base, uint64_t dst_elems, void* stream) {
  if (!nz) return -1;
  if (num == 0) return 0;
  if (!specs || !dst) return -1;
  for (uint32_t t = 0; t < num; ++t)
    if (specs[t].offset < base || specs[t].offset - base + (uint64_t)specs[t].K * specs[t].N > dst_elems)
      return -2;
  hipStream_t st = (hipStream_t)stream;
  const uint32_t chunk = 32768;  // grid.y limit: fill in slices of series
  syn_series* d_specs = nullptr;
  const uint32_t cap = num < chunk ? num : chunk;
  if (hipMalloc(&d_specs, sizeof(syn_series) * cap) != hipSuccess) return -3;
  int rc = 0;
  for (uint32_t s0 = 0; s0 < num && !rc; s0 += chunk) {
    const uint32_t n = (num - s0) < chunk ? (num - s0) : chunk;
    if (hipMemcpyAsync(d_specs, specs + s0, sizeof(syn_series) * n, hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = -3;
      break;
    }
    hipLaunchKernelGGL(fill_kernel, dim3(64, n), dim3(256), 0, st, d_specs, *nz, seed, dst, base);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = -3;
  }
  hipFree(d_specs);
  return rc;
}

// Raw Philox4x32-10 block, exposed for known-answer tests of the generator.
void syn_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const u4 r = philox4x32_10(u4{ctr[0], ctr[1], ctr[2], ctr[3]}, key[0], key[1]);
  out[0] = r.x;
  out[1] = r.y;
  out[2] = r.z;
  out[3] = r.w;
}

// The generator's scalar math, exposed for accuracy tests.
double syn_math(int which, double x) {
  switch (which) {
    case 0: return syn_exp(x);
    case 1: return syn_log(x);
    case 2: return syn_cos2pi(x);
    default: return 0.0;
  }
}

}  // extern "C"

// Proposal network kernels: 1-D convolutions on BF16 MFMA with FP32
// accumulation, the weight-gradient reduction, softmax cross-entropy, the
// proposal (argmax + window mass) and Adam.
//
// Row layout. A batch of B series is one long sequence of B * SR rows
// (SR = roundup(max_K + 4, 16)); series s owns rows [s SR + 2, s SR + 2 + K_s)
// and every other row of its slot is kept zero, so the zero padding of each
// kernel-5 convolution at the series' ends is simply the neighbouring zero
// rows and every layer is one convolution over the whole sequence.
//
// A layer y[t][o] = b[o] + sum_{k<5, i<CIN} W[o][i][k] x[t + k - 2][i] is an
// implicit GEMM with M = rows (16 per MFMA tile), N = output channels and
// reduction index j = k * CIN + i (32 per v_mfma_f32_16x16x32_bf16). The
// input gradient of a layer is the same convolution of the output gradient
// with W'[i][o][k] = W[o][i][4 - k], so one kernel serves both directions.
#pragma once

#include "ks.h"
#include "ks_wave.hpp"

namespace ks {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int KW = 5;
constexpr int TM = 64;   // rows per tile: four waves of 16
constexpr int NTC = 256;

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ float relu(float v) { return v > 0.0f ? v : 0.0f; }

// Row `row` holds data iff it lies inside its series' rows.
__device__ __forceinline__ bool row_valid(uint64_t row, uint64_t rows, uint32_t SR, const uint32_t* __restrict__ Ks) {
  if (row >= rows) return false;
  const uint64_t s = row / SR;
  const uint32_t r = (uint32_t)(row - s * SR);
  return r >= 2 && r - 2 < Ks[s];
}

__device__ __forceinline__ f32x4 mfma16(const u32x4& a, const u32x4& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0,
                                                 0, 0);
}

enum Epi { EPI_RELU = 0, EPI_LOGIT = 1, EPI_BWD = 2 };

template <int CIN, int COUT>
struct ConvShape {
  static constexpr int J = KW * CIN;             // reduction length
  static constexpr int JP = (J + 31) / 32 * 32;  // padded to whole MFMA steps
  static constexpr int WST = JP + 8;             // LDS row stride of weights (bf16)
  static constexpr int XST = CIN + 8;            // LDS row stride of the input tile
  static constexpr int XR = TM + 4;              // input rows per tile (2-row halo each side)
  static constexpr int NQ = JP / 32;
  static constexpr int NN = COUT / 16;
};

// One convolution over `rows` rows.
//   X     [rows][CIN]  bf16 input
//   Wg    [COUT][5 CIN] bf16 weights, j = k CIN + i
//   bias  [COUT] fp32 (EPI_RELU / EPI_LOGIT)
//   EPI_RELU   Y[row][o] = bf16(relu(acc + b)) on valid rows, 0 elsewhere
//   EPI_LOGIT  Yf[row]   = acc[o=0] + b[0] on valid rows, 0 elsewhere
//   EPI_BWD    d = acc where Mask[row][o] != 0 (the layer input was > 0) and the
//              row is valid, else 0: Y[row][o] = bf16(d), Yf[row][o] = d
template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(NTC) void conv_kernel(const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wg,
                                                   const float* __restrict__ bias, uint64_t rows, uint32_t SR,
                                                   const uint32_t* __restrict__ Ks, uint16_t* __restrict__ Y,
                                                   float* __restrict__ Yf, const uint16_t* __restrict__ Mask) {
  using S = ConvShape<CIN, COUT>;
  __shared__ __align__(16) uint16_t wl[COUT * S::WST];
  __shared__ __align__(16) uint16_t xl[S::XR * S::XST];
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = wave_id();
  for (uint32_t q = tid; q < (uint32_t)(COUT * S::JP); q += NTC) {
    const uint32_t o = q / S::JP, j = q - o * S::JP;
    wl[o * S::WST + j] = j < (uint32_t)S::J ? Wg[o * S::J + j] : (uint16_t)0;
  }
  const uint32_t m = lane & 15u, kg = lane >> 4;
  const uint64_t ntiles = (rows + TM - 1) / TM;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = (int64_t)(tile * TM);
    __syncthreads();
    for (uint32_t q = tid; q < (uint32_t)(S::XR * CIN); q += NTC) {
      const uint32_t rr = q / CIN, i = q - rr * CIN;
      const int64_t row = r0 - 2 + (int64_t)rr;
      xl[rr * S::XST + i] = (row >= 0 && (uint64_t)row < rows) ? X[(uint64_t)row * CIN + i] : (uint16_t)0;
    }
    __syncthreads();
    f32x4 acc[S::NN];
#pragma unroll
    for (int n = 0; n < S::NN; ++n) acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < S::NQ; ++q) {
      const int j0 = q * 32 + (int)kg * 8;
      u32x4 a = u32x4{0u, 0u, 0u, 0u};
      if (j0 < S::J) {
        const int k = j0 / CIN, i0 = j0 - k * CIN;
        // tile row w*16 + m sits at xl row w*16 + m + 2; tap k reads row + k - 2
        a = *reinterpret_cast<const u32x4*>(&xl[(w * 16 + m + k) * S::XST + i0]);
      }
#pragma unroll
      for (int n = 0; n < S::NN; ++n) {
        const u32x4 b = *reinterpret_cast<const u32x4*>(&wl[(n * 16 + m) * S::WST + j0]);
        acc[n] = mfma16(a, b, acc[n]);
      }
    }
#pragma unroll
    for (int n = 0; n < S::NN; ++n) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t row = (uint64_t)r0 + w * 16 + kg * 4 + e;
        if (row >= rows) continue;
        const uint32_t o = n * 16 + m;
        const bool valid = row_valid(row, rows, SR, Ks);
        if (EPI == EPI_RELU) {
          Y[row * COUT + o] = valid ? f2bf(relu(acc[n][e] + bias[o])) : (uint16_t)0;
        } else if (EPI == EPI_LOGIT) {
          if (o == 0) Yf[row] = valid ? acc[n][e] + bias[0] : 0.0f;
        } else {
          const float d = (valid && Mask[row * COUT + o] != 0) ? acc[n][e] : 0.0f;
          Y[row * COUT + o] = f2bf(d);
          Yf[row * COUT + o] = d;
        }
      }
    }
  }
}

// ------------------------------------------------------------ fused forward
// The whole network over tiles of FT rows, for inference. Tiles follow the
// series: tile f of series s starts at its row f FT (slot row s SR + 2 + f FT),
// for f < ceil(K / FT), so no tile is spent on a slot's padding, and a tile
// writes the logits of its own series' rows only (the padding's logits are
// never read). A tile's frame is its FT rows plus FH = 8 halo rows on each
// side (2 per layer): frame row f is slot row r0 - FH + f. Every layer
// computes all FR = FT + 16 frame rows (nine 16-row MFMA blocks); the rows
// within 2l of the frame's ends are wrong after layer l (their inputs fall off
// the frame) but never reach the rows [FH, FH + FT) whose logits are written. Activations stay in LDS as bf16,
// zeroed on rows outside their series exactly as the per-layer kernels write
// them, and each output accumulates over j in the per-layer kernels' order
// (same MFMA steps, bias added last). Wave w owns output channels 16w .. 16w + 15
// of layers 0..2 and keeps their weights in registers for the whole launch.
constexpr int FT = 128;
constexpr int FH = 8;
constexpr int FR = FT + 2 * FH;  // 144
constexpr int FBLK = FR / 16;    // 9 row blocks
constexpr int FST = 64 + 8;      // LDS row stride of a 64-channel activation buffer (bf16)
constexpr int FXS = 16 + 8;      // LDS row stride of the 16-channel input buffer
constexpr int FW3 = 320 + 8;     // LDS row stride of the last layer's weights

struct FusedSmem {
  uint16_t act[2][(FR + 4) * FST];  // buffer row f + 2 holds frame row f; rows 0, 1, FR + 2, FR + 3 stay zero
  uint16_t x[(FR + 4) * FXS];
  uint16_t w3[2 * FW3];             // row 0: W3[0][j]; row 1: zeros (output channels 1..15)
  uint64_t valid[4];                // bit f % 64 of word f / 64: frame row f lies inside a series
};

// Bits 4 b + e (b < FBLK, e < 4) of a lane's row mask: frame row 16 b + 4 kg + e
// is valid (the rows whose outputs this lane holds in an MFMA result).
__device__ __forceinline__ uint64_t fused_lane_rows(const uint64_t (&v)[3], uint32_t kg) {
  uint64_t m = 0;
#pragma unroll
  for (int b = 0; b < FBLK; ++b) {
    const int f0 = 16 * b;  // + 4 kg
    const uint64_t word = v[f0 / 64];
    m |= ((word >> ((f0 % 64) + 4 * kg)) & 0xFull) << (4 * b);
  }
  return m;
}

// One 64-output-channel layer over the frame for this wave's 16 channels:
// out[f][16 w + m] = bf16(relu(b + sum_j W[16 w + m][j] in[f + k - 2][i])) on
// valid rows, 0 elsewhere (j = k CIN + i).
template <int CIN, int NQ>
__device__ __forceinline__ void fused_layer(const uint16_t* __restrict__ in, int ist, const u32x4 (&B)[NQ],
                                            float bias, uint16_t* __restrict__ out, uint64_t rows,
                                            uint32_t w, uint32_t m, uint32_t kg) {
  constexpr int J = KW * CIN;
#pragma unroll 1
  for (int g = 0; g < FBLK; g += 3) {
    f32x4 acc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // A operands one k-step ahead of the MFMAs; the scheduling barrier keeps
    // the compiler from hoisting every step's loads (and their registers)
    auto load_a = [&](int q, u32x4 (&a)[3]) {
      const int j0 = q * 32 + (int)kg * 8;
      const int k = j0 / CIN, i0 = j0 - k * CIN;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        // frame row 16 (g + t) + m, tap k: buffer row 16 (g + t) + m + k
        a[t] = (NQ * 32 <= J || j0 < J) ? *reinterpret_cast<const u32x4*>(&in[((g + t) * 16 + (int)m + k) * ist + i0])
                                        : u32x4{0u, 0u, 0u, 0u};
      }
    };
    u32x4 a0[3], a1[3];
    load_a(0, a0);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      u32x4(&cur)[3] = (q & 1) ? a1 : a0;
      u32x4(&nxt)[3] = (q & 1) ? a0 : a1;
      if (q + 1 < NQ) load_a(q + 1, nxt);
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[t] = mfma16(cur[t], B[q], acc[t]);
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int f = (g + t) * 16 + (int)kg * 4 + e;
        const bool v = (rows >> (4 * (g + t) + e)) & 1u;
        out[(f + 2) * FST + w * 16 + m] = v ? f2bf(relu(acc[t][e] + bias)) : (uint16_t)0;
      }
  }
}

// x0 [rows][16] bf16 (channels 11..15 zero), wf[l] as for conv_kernel,
// logits [rows] fp32 (0 on rows outside every series).
__global__ __launch_bounds__(NTC) __attribute__((amdgpu_waves_per_eu(3))) void fused_forward_kernel(const uint16_t* __restrict__ x0, uint64_t rows,
                                                            uint32_t SR, const uint32_t* __restrict__ Ks,
                                                            uint32_t num_series, uint32_t tiles_per_series,
                                                            const uint16_t* __restrict__ w0,
                                                            const uint16_t* __restrict__ w1,
                                                            const uint16_t* __restrict__ w2,
                                                            const uint16_t* __restrict__ w3,
                                                            const float* __restrict__ b0, const float* __restrict__ b1,
                                                            const float* __restrict__ b2, const float* __restrict__ b3,
                                                            float* __restrict__ logits) {
  __shared__ __align__(16) FusedSmem sm;
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const uint32_t m = lane & 15u, kg = lane >> 4;
  const uint32_t o = w * 16 + m;
  // B operands of this wave's channels: W[o][32 q + 8 kg .. + 7]; layers 1 and
  // 2 stay in registers, layer 0's (three k-steps) are read again per tile
  u32x4 B1[10], B2[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    B1[q] = *reinterpret_cast<const u32x4*>(w1 + o * 320 + q * 32 + kg * 8);
    B2[q] = *reinterpret_cast<const u32x4*>(w2 + o * 320 + q * 32 + kg * 8);
  }
  const float bias0 = b0[o], bias1 = b1[o], bias2 = b2[o], bias3 = b3[0];
  for (uint32_t q = tid; q < 2u * FW3; q += NTC) sm.w3[q] = q < 320u ? w3[q] : (uint16_t)0;
  for (uint32_t q = tid; q < 4u * FST; q += NTC) {
    const uint32_t r = q / FST, c = q - r * FST, br = r < 2 ? r : FR + r;
    sm.act[0][br * FST + c] = 0;
    sm.act[1][br * FST + c] = 0;
  }
  for (uint32_t q = tid; q < 4u * FXS; q += NTC) {
    const uint32_t r = q / FXS, c = q - r * FXS, br = r < 2 ? r : FR + r;
    sm.x[br * FXS + c] = 0;
  }
  const uint64_t ntiles = (uint64_t)num_series * tiles_per_series;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const uint32_t ser = (uint32_t)(tile / tiles_per_series);
    const uint32_t t0 = (uint32_t)(tile - (uint64_t)ser * tiles_per_series) * FT;  // the tile's first row in its series
    const uint32_t K = Ks[ser];
    if (t0 >= K) continue;  // past the series' last row (block-uniform)
    const uint64_t sbase = (uint64_t)ser * SR + 2;
    const int64_t r0 = (int64_t)(sbase + t0);
    __syncthreads();
    // frame row f = tid (FR <= NTC): its validity as one bit per row, by ballot
    const int64_t vrow = r0 - FH + (int64_t)tid;
    const bool v = tid < (uint32_t)FR && vrow >= 0 && row_valid((uint64_t)vrow, rows, SR, Ks);
    const uint64_t vb = ballot(v);
    if (lane == 0) sm.valid[w] = vb;  // read after the barrier below
    for (uint32_t q = tid; q < 2u * FR; q += NTC) {
      const uint32_t f = q >> 1, h = q & 1u;
      const int64_t row = r0 - FH + (int64_t)f;
      u32x4 v = u32x4{0u, 0u, 0u, 0u};
      if (row >= 0 && (uint64_t)row < rows) v = *reinterpret_cast<const u32x4*>(x0 + (uint64_t)row * 16 + h * 8);
      *reinterpret_cast<u32x4*>(&sm.x[(f + 2) * FXS + h * 8]) = v;
    }
    __syncthreads();
    const uint64_t vw[3] = {sm.valid[0], sm.valid[1], sm.valid[2]};
    const uint64_t lrows = fused_lane_rows(vw, kg);
    u32x4 B0[3];
    {
      const uint16_t* w0p = w0;
      asm volatile("" : "+v"(w0p));  // read per tile: keeps the compiler from pinning B0 in registers
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const int j0 = q * 32 + (int)kg * 8;
        B0[q] = j0 < 80 ? *reinterpret_cast<const u32x4*>(w0p + o * 80 + j0) : u32x4{0u, 0u, 0u, 0u};
      }
    }
    fused_layer<16, 3>(sm.x, FXS, B0, bias0, sm.act[0], lrows, w, m, kg);
    __syncthreads();
    fused_layer<64, 10>(sm.act[0], FST, B1, bias1, sm.act[1], lrows, w, m, kg);
    __syncthreads();
    fused_layer<64, 10>(sm.act[1], FST, B2, bias2, sm.act[0], lrows, w, m, kg);
    __syncthreads();
    // last layer (one output channel): wave w takes row blocks w, w + 4, w + 8
    const uint16_t* w3row = &sm.w3[m == 0 ? 0 : FW3];
    for (int blk = (int)w; blk < FBLK; blk += 4) {
      f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
      auto load_ab = [&](int q, u32x4& a, u32x4& b) {
        const int j0 = q * 32 + (int)kg * 8;
        const int k = j0 / 64, i0 = j0 - k * 64;
        a = *reinterpret_cast<const u32x4*>(&sm.act[0][(blk * 16 + (int)m + k) * FST + i0]);
        b = *reinterpret_cast<const u32x4*>(&w3row[j0]);
      };
      u32x4 a0, b0, a1, b1;
      load_ab(0, a0, b0);
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        u32x4& ca = (q & 1) ? a1 : a0;
        u32x4& cb = (q & 1) ? b1 : b0;
        if (q + 1 < 10) load_ab(q + 1, (q & 1) ? a0 : a1, (q & 1) ? b0 : b1);
        acc = mfma16(ca, cb, acc);
        __builtin_amdgcn_sched_barrier(0);
      }
      if (m == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int f = blk * 16 + (int)kg * 4 + e;
          const int64_t row = r0 - FH + f;
          if (f >= FH && f < FH + FT && (uint64_t)row - sbase < K) logits[row] = acc[e] + bias3;
        }
      }
    }
  }
}

// Weight gradient partials of one layer:
//   dW[o][j] = sum_rows dY[row][o] X[row + k - 2][i]   (j = k CIN + i)
//   db[o]    = sum_rows dYf[row][o]
// as a GEMM with M = output channels, N = j, reduction over rows. Workgroup g
// accumulates its tiles and writes part[g][o * J + j] and part[g][COUT*J + o].
template <int CIN, int COUT>
struct DwShape {
  static constexpr int J = KW * CIN;
  static constexpr int NM = COUT / 16;
  static constexpr int NJ = J / 16;
  static constexpr int TILES = NM * NJ;
  static constexpr int PER_WAVE = (TILES + 3) / 4;
  static constexpr int YST = TM + 8;   // LDS stride of dY^T rows (bf16)
  static constexpr int XST = TM + 12;  // LDS stride of X^T rows (bf16): TM + 4 halo + pad
  static constexpr int PART = COUT * J + COUT;
};

template <int CIN, int COUT>
__global__ __launch_bounds__(NTC) void dw_kernel(const uint16_t* __restrict__ dY, const float* __restrict__ dYf,
                                                 const uint16_t* __restrict__ X, uint64_t rows,
                                                 float* __restrict__ part) {
  using S = DwShape<CIN, COUT>;
  __shared__ __align__(16) uint16_t yt[COUT * S::YST];
  __shared__ __align__(16) uint16_t xt[CIN * S::XST];
  const uint32_t tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const uint32_t m = lane & 15u, kg = lane >> 4;
  f32x4 acc[S::PER_WAVE];
#pragma unroll
  for (int t = 0; t < S::PER_WAVE; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  float db = 0.0f;  // thread tid < COUT: bias gradient of channel tid
  const uint64_t ntiles = (rows + TM - 1) / TM;
  for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t r0 = (int64_t)(tile * TM);
    __syncthreads();
    for (uint32_t q = tid; q < (uint32_t)(TM * COUT); q += NTC) {
      const uint32_t rr = q / COUT, o = q - rr * COUT;
      const uint64_t row = (uint64_t)r0 + rr;
      yt[o * S::YST + rr] = row < rows ? dY[row * COUT + o] : (uint16_t)0;
    }
    for (uint32_t q = tid; q < (uint32_t)((TM + 4) * CIN); q += NTC) {
      const uint32_t rr = q / CIN, i = q - rr * CIN;
      const int64_t row = r0 - 2 + (int64_t)rr;
      xt[i * S::XST + rr] = (row >= 0 && (uint64_t)row < rows) ? X[(uint64_t)row * CIN + i] : (uint16_t)0;
    }
    if (tid < (uint32_t)COUT)
      for (uint32_t rr = 0; rr < (uint32_t)TM; ++rr) {
        const uint64_t row = (uint64_t)r0 + rr;
        if (row < rows) db += dYf[row * COUT + tid];
      }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < S::PER_WAVE; ++t) {
      const int tt = w * S::PER_WAVE + t;
      if (tt >= S::TILES) break;
      const int mt = tt / S::NJ, nt = tt - mt * S::NJ;
      const uint32_t o = mt * 16 + m;
      const uint32_t j = nt * 16 + m;
      const uint32_t k = j / CIN, i = j - k * CIN;
#pragma unroll
      for (int q = 0; q < TM / 32; ++q) {
        const uint32_t rr = q * 32 + kg * 8;
        const u32x4 a = *reinterpret_cast<const u32x4*>(&yt[o * S::YST + rr]);
        // X[r0 + rr + e + k - 2] = xt[i][rr + e + k]: 8 bf16 at an odd offset when k is odd
        uint32_t bw[4];
#pragma unroll
        for (int e = 0; e < 4; ++e)
          bw[e] = (uint32_t)xt[i * S::XST + rr + k + 2 * e] | ((uint32_t)xt[i * S::XST + rr + k + 2 * e + 1] << 16);
        acc[t] = mfma16(a, u32x4{bw[0], bw[1], bw[2], bw[3]}, acc[t]);
      }
    }
  }
  float* out = part + (uint64_t)blockIdx.x * S::PART;
#pragma unroll
  for (int t = 0; t < S::PER_WAVE; ++t) {
    const int tt = w * S::PER_WAVE + t;
    if (tt >= S::TILES) break;
    const int mt = tt / S::NJ, nt = tt - mt * S::NJ;
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(mt * 16 + kg * 4 + e) * S::J + nt * 16 + m] = acc[t][e];
  }
  if (tid < (uint32_t)COUT) out[COUT * S::J + tid] = db;
}

// grad[p] = sum over g < G of part[g][p], p < n.
__global__ __launch_bounds__(NTC) void reduce_parts_kernel(const float* __restrict__ part, uint32_t G, uint32_t n,
                                                           float* __restrict__ grad) {
  const uint32_t p = blockIdx.x * NTC + threadIdx.x;
  if (p >= n) return;
  float s = 0.0f;
  for (uint32_t g = 0; g < G; ++g) s += part[(uint64_t)g * n + p];
  grad[p] = s;
}

// ---------------------------------------------------------------- parameters
//
// Master vector (fp32, 44993): W0[64][11][5] b0[64] W1[64][64][5] b1[64]
// W2[64][64][5] b2[64] W3[1][64][5] b3[1]. Input channels of layer 0: the nine
// decile features, then t / (K-1) and 4 t (K - t) / K^2.
struct Layer {
  int cin, cout, cin_pad, cout_pad;
  uint32_t w_off, b_off;
};
__device__ __host__ inline Layer layer_info(int l) {
  switch (l) {
    case 0: return Layer{11, 64, 16, 64, 0u, 3520u};
    case 1: return Layer{64, 64, 64, 64, 3584u, 24064u};
    case 2: return Layer{64, 64, 64, 64, 24128u, 44608u};
    default: return Layer{64, 1, 64, 16, 44672u, 44992u};
  }
}
constexpr uint32_t kNumParams = 44993;

// Position channels of row t of a K-row series (double, rounded to float).
__device__ __forceinline__ float pos_frac(uint32_t t, uint32_t K) {
  return (float)((double)t / (double)(K > 1 ? K - 1 : 1));
}
__device__ __forceinline__ float pos_centre(uint32_t t, uint32_t K) {
  return (float)(4.0 * (double)t * (double)(K - t) / ((double)K * (double)K));
}

// Entries of all shadow copies (forward weights and biases of every layer).
constexpr uint32_t kShadowEntries = (64 * 5 * 16 + 64) + 2 * (64 * 5 * 64 + 64) + (16 * 5 * 64 + 16);

// Device copies used by the kernels.
struct Shadow {
  uint16_t* wf[4];  // forward: [cout_pad][5 cin_pad], j = k cin_pad + i
  uint16_t* wb[4];  // backward data (l >= 1): [cin_pad][5 cout_pad], j = k cout_pad + o, tap flipped
  float* b[4];      // [cout_pad]
};

// Rebuild every shadow copy from the master vector (one thread per entry).
__global__ __launch_bounds__(NTC) void shadow_kernel(const float* __restrict__ theta, Shadow sh) {
  const uint32_t t = blockIdx.x * NTC + threadIdx.x;
  uint32_t base = 0;
  for (int l = 0; l < 4; ++l) {
    const Layer L = layer_info(l);
    const uint32_t nf = (uint32_t)(L.cout_pad * KW * L.cin_pad);
    if (t >= base && t < base + nf) {
      const uint32_t q = t - base, o = q / (KW * L.cin_pad), j = q - o * (KW * L.cin_pad);
      const uint32_t k = j / L.cin_pad, i = j - k * L.cin_pad;
      const float v = ((int)o < L.cout && (int)i < L.cin) ? theta[L.w_off + (o * L.cin + i) * KW + k] : 0.0f;
      sh.wf[l][q] = f2bf(v);
      if (l >= 1) {
        // wb[i][k' cout_pad + o] = W[o][i][4 - k']
        const uint32_t kp = KW - 1 - k;
        sh.wb[l][i * (KW * L.cout_pad) + kp * L.cout_pad + o] = f2bf(v);
      }
    }
    base += nf;
    if (t >= base && t < base + (uint32_t)L.cout_pad) {
      const uint32_t o = t - base;
      sh.b[l][o] = (int)o < L.cout ? theta[L.b_off + o] : 0.0f;
    }
    base += L.cout_pad;
  }
}

// Adam (Kingma & Ba) on the master vector; gradients gathered from the
// per-layer reduced partials ([cout_pad][5 cin_pad] then [cout_pad] biases).
__global__ __launch_bounds__(NTC) void adam_kernel(float* __restrict__ theta, float* __restrict__ mom1,
                                                   float* __restrict__ mom2, float* __restrict__ grad_out,
                                                   const float* __restrict__ g0, const float* __restrict__ g1,
                                                   const float* __restrict__ g2, const float* __restrict__ g3,
                                                   float lr, float bc1, float bc2, int apply) {
  const uint32_t p = blockIdx.x * NTC + threadIdx.x;
  if (p >= kNumParams) return;
  int l = 3;
  for (int q = 0; q < 4; ++q) {
    const Layer L = layer_info(q);
    if (p < L.b_off + (uint32_t)L.cout) {
      l = q;
      break;
    }
  }
  const Layer L = layer_info(l);
  const float* g = l == 0 ? g0 : (l == 1 ? g1 : (l == 2 ? g2 : g3));
  const uint32_t J = KW * L.cin_pad;
  float gv;
  if (p < L.b_off) {
    const uint32_t q = p - L.w_off, o = q / (L.cin * KW), r = q - o * (L.cin * KW), i = r / KW, k = r - i * KW;
    gv = g[o * J + k * L.cin_pad + i];
  } else {
    gv = g[L.cout_pad * J + (p - L.b_off)];
  }
  grad_out[p] = gv;
  if (!apply) return;
  const float m = 0.9f * mom1[p] + 0.1f * gv;
  const float v = 0.999f * mom2[p] + 0.001f * gv * gv;
  mom1[p] = m;
  mom2[p] = v;
  theta[p] -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
}

// p[i] = 0 for i < n (a plain fill kernel rather than a memset node, so that a
// captured graph replays it like any other kernel).
__global__ __launch_bounds__(NTC) void zero_kernel(float* __restrict__ p, uint32_t n) {
  const uint32_t i = blockIdx.x * NTC + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// ---------------------------------------------------------------- series heads

// Number of labels >= 1 in the batch (the series that enter the loss).
__global__ __launch_bounds__(NTC) void count_labels_kernel(const int32_t* __restrict__ labels, uint32_t n,
                                                           uint32_t* __restrict__ count) {
  __shared__ uint32_t c;
  if (threadIdx.x == 0) c = 0;
  __syncthreads();
  uint32_t local = 0;
  for (uint32_t s = threadIdx.x; s < n; s += NTC) local += labels[s] >= 1 ? 1u : 0u;
  atomicAdd(&c, local);
  __syncthreads();
  if (threadIdx.x == 0) *count = c;
}

// Softmax over rows t = 1..K-1 of each series (one wave per series).
// Training (labels != null): loss += -log p[label] / B_sig and dlogit rows
// (bf16 + fp32, 16 channels, channel 0 used) = (p - onehot) / B_sig on rows
// 1..K-1 of series with label >= 1, zero elsewhere. Inference: proposal =
// argmax (smallest row on ties), confidence = softmax mass of rows within
// +-w of it.
__global__ __launch_bounds__(NTC) void softmax_kernel(const float* __restrict__ logits, uint32_t num_series,
                                                      uint32_t SR, const uint32_t* __restrict__ Ks,
                                                      const int32_t* __restrict__ labels,
                                                      const uint32_t* __restrict__ nsig, float* __restrict__ loss,
                                                      uint16_t* __restrict__ dY, float* __restrict__ dYf, uint32_t w,
                                                      int32_t* __restrict__ proposal, float* __restrict__ conf) {
  const uint32_t lane = lane_id();
  const uint32_t s = blockIdx.x * (NTC / kWave) + wave_id();
  if (s >= num_series) return;
  const uint32_t K = Ks[s];
  const uint64_t base = (uint64_t)s * SR + 2;
  if (K < 2) {
    if (proposal && lane == 0) {
      proposal[s] = 0;
      conf[s] = 0.0f;
    }
    if (dY)
      for (uint32_t r = lane; r < SR; r += kWave)
        for (int c = 0; c < 16; ++c) {
          dY[((uint64_t)s * SR + r) * 16 + c] = 0;
          dYf[((uint64_t)s * SR + r) * 16 + c] = 0.0f;
        }
    return;
  }
  // max and argmax over t = 1..K-1
  float mx = -3.402823466e38f;
  uint32_t am = 0xffffffffu;
  for (uint32_t t = 1 + lane; t < K; t += kWave) {
    const float z = logits[base + t];
    if (z > mx || (z == mx && t < am)) {
      mx = z;
      am = t;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const float zm = __shfl_xor(mx, o);
    const uint32_t ta = (uint32_t)__shfl_xor((int)am, o);
    if (zm > mx || (zm == mx && ta < am)) {
      mx = zm;
      am = ta;
    }
  }
  float sum = 0.0f;
  for (uint32_t t = 1 + lane; t < K; t += kWave) sum += __expf(logits[base + t] - mx);
  for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o);
  if (proposal) {
    const uint32_t lo = am > w ? am - w : 1u, hi = min(K - 1, am + w);
    float part = 0.0f;
    for (uint32_t t = lo + lane; t <= hi; t += kWave) part += __expf(logits[base + t] - mx);
    for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o);
    if (lane == 0) {
      proposal[s] = (int32_t)am;
      conf[s] = part / sum;
    }
  }
  if (dY) {
    const int32_t lab = labels[s];
    const bool use = lab >= 1 && (uint32_t)lab < K;
    const float inv = 1.0f / (float)max(*nsig, 1u);
    for (uint32_t r = lane; r < SR; r += kWave) {
      const uint64_t row = (uint64_t)s * SR + r;
      float d = 0.0f;
      if (use && r >= 3 && r - 2 < K) {
        const uint32_t t = r - 2;
        d = (__expf(logits[base + t] - mx) / sum - (t == (uint32_t)lab ? 1.0f : 0.0f)) * inv;
      }
      dY[row * 16] = f2bf(d);
      dYf[row * 16] = d;
      for (int c = 1; c < 16; ++c) {
        dY[row * 16 + c] = 0;
        dYf[row * 16 + c] = 0.0f;
      }
    }
    if (use && lane == 0) atomicAdd(loss, (logf(sum) - (logits[base + lab] - mx)) * inv);
  }
}

// Proposal without the network: the row after the largest jump of the per-row
// median (feature 5, the fifth decile), |f_t - f_(t-1)| in FP64 (exact for
// floats), ties to the smaller row; confidence 1 (always refined). One wave per
// series, features from the feature pass's slot rows.
__global__ __launch_bounds__(NTC) void median_jump_kernel(const float* __restrict__ feat, uint32_t num_series,
                                                          uint32_t SR, const uint32_t* __restrict__ Ks,
                                                          int32_t* __restrict__ proposal,
                                                          float* __restrict__ conf) {
  const uint32_t lane = lane_id();
  const uint32_t s = blockIdx.x * (NTC / kWave) + wave_id();
  if (s >= num_series) return;
  const uint32_t K = Ks[s];
  const uint64_t base = (uint64_t)s * SR + 2;
  double best = -1.0;
  uint32_t arg = 0;
  for (uint32_t t = 1 + lane; t < K; t += kWave) {
    const double j = fabs((double)feat[(base + t) * 9 + 4] - (double)feat[(base + t - 1) * 9 + 4]);
    if (j > best) {  // t grows within a lane: the first maximum is kept
      best = j;
      arg = t;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const double bo = __shfl_xor(best, o);
    const uint32_t ao = (uint32_t)__shfl_xor((int)arg, o);
    if (bo > best || (bo == best && ao < arg && ao != 0)) {
      best = bo;
      arg = ao;
    }
  }
  if (lane == 0) {
    proposal[s] = K >= 2 ? (int32_t)arg : 0;
    conf[s] = K >= 2 ? 1.0f : 0.0f;
  }
}

// Caller features (fp32 [rows at aux_offset][9]) -> network input rows
// (bf16, 16 channels) in the slot layout, plus each series' K (0 if invalid).
__global__ __launch_bounds__(NTC) void pack_features_kernel(const float* __restrict__ feat, uint64_t feat_rows,
                                                            const ks_desc* __restrict__ desc, uint32_t num_series,
                                                            uint32_t max_K, uint32_t SR,
                                                            uint16_t* __restrict__ x0,
                                                            uint32_t* __restrict__ Ks) {
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const bool ok = d.K >= 2 && d.K <= max_K && d.aux_offset <= feat_rows && d.K <= feat_rows - d.aux_offset;
  const uint32_t K = ok ? d.K : 0u;
  for (uint32_t q = threadIdx.x; q < SR * 16; q += NTC) {
    const uint32_t r = q / 16, k = q - r * 16;
    uint16_t b = 0;
    if (r >= 2 && r - 2 < K) {
      if (k < 9)
        b = f2bf(feat[(d.aux_offset + r - 2) * 9 + k]);
      else if (k == 9)
        b = f2bf(pos_frac(r - 2, K));
      else if (k == 10)
        b = f2bf(pos_centre(r - 2, K));
    }
    x0[((uint64_t)s * SR + r) * 16 + k] = b;
  }
  if (threadIdx.x == 0) Ks[s] = K;
}

// Caller logit gradients (fp32 rows aux_offset + t) -> the backward pass's
// input in the slot layout: bf16 and fp32 copies of channel 0 (16 channels, the
// others zero), zero on rows outside every series.
__global__ __launch_bounds__(NTC) void pack_dlogits_kernel(const float* __restrict__ dz, uint64_t dz_rows,
                                                           const ks_desc* __restrict__ desc, uint32_t num_series,
                                                           uint32_t SR, const uint32_t* __restrict__ Ks,
                                                           uint16_t* __restrict__ dY, float* __restrict__ dYf) {
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  uint32_t K = Ks[s];
  if (!(d.aux_offset <= dz_rows && K <= dz_rows - d.aux_offset)) K = 0;
  for (uint32_t q = threadIdx.x; q < SR * 16; q += NTC) {
    const uint32_t r = q / 16, c = q - r * 16;
    const float v = (c == 0 && r >= 2 && r - 2 < K) ? dz[d.aux_offset + r - 2] : 0.0f;
    dY[((uint64_t)s * SR + r) * 16 + c] = f2bf(v);
    dYf[((uint64_t)s * SR + r) * 16 + c] = v;
  }
}

// Per-layer values of one forward (and backward) pass -> caller rows
// aux_offset + t, as floats: acts row = x0[11] a1[64] a2[64] a3[64] logit
// (KS_CNN_TRACE_ACTS), gin row = dlogit, then the gradients at y2, y1, y0
// [64 each] (KS_CNN_TRACE_GRADS). dyf0 == nullptr: no backward values.
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ __launch_bounds__(NTC) void trace_copy_kernel(const ks_desc* __restrict__ desc, uint32_t num_series,
                                                         uint32_t SR, const uint32_t* __restrict__ Ks,
                                                         const uint16_t* __restrict__ x0,
                                                         const uint16_t* __restrict__ a1,
                                                         const uint16_t* __restrict__ a2,
                                                         const uint16_t* __restrict__ a3,
                                                         const float* __restrict__ logits,
                                                         const float* __restrict__ dz, const float* __restrict__ dyf0,
                                                         const float* __restrict__ dyf1, const float* __restrict__ dyf2,
                                                         float* __restrict__ acts, float* __restrict__ gin,
                                                         uint64_t out_rows) {
  constexpr uint32_t NA = 11 + 3 * 64 + 1, NG = 1 + 3 * 64;
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const uint32_t K = Ks[s];
  if (!(d.aux_offset <= out_rows && K <= out_rows - d.aux_offset)) return;
  for (uint32_t q = threadIdx.x; q < K * NA && acts; q += NTC) {
    const uint32_t t = q / NA, c = q - t * NA;
    const uint64_t row = (uint64_t)s * SR + 2 + t;
    float v;
    if (c < 11) v = bf2f(x0[row * 16 + c]);
    else if (c < 75) v = bf2f(a1[row * 64 + (c - 11)]);
    else if (c < 139) v = bf2f(a2[row * 64 + (c - 75)]);
    else if (c < 203) v = bf2f(a3[row * 64 + (c - 139)]);
    else v = logits[row];
    acts[(d.aux_offset + t) * NA + c] = v;
  }
  for (uint32_t q = threadIdx.x; q < K * NG && gin && dyf0; q += NTC) {
    const uint32_t t = q / NG, c = q - t * NG;
    const uint64_t row = (uint64_t)s * SR + 2 + t;
    float v;
    if (c == 0) v = dz[row * 16];
    else if (c < 65) v = dyf0[row * 64 + (c - 1)];
    else if (c < 129) v = dyf1[row * 64 + (c - 65)];
    else v = dyf2[row * 64 + (c - 129)];
    gin[(d.aux_offset + t) * NG + c] = v;
  }
}

// Logits in the slot layout -> caller rows (aux_offset + t), nullable output.
__global__ __launch_bounds__(NTC) void unpack_logits_kernel(const float* __restrict__ lg, const ks_desc* __restrict__ desc,
                                                            uint32_t num_series, uint32_t SR,
                                                            const uint32_t* __restrict__ Ks, float* __restrict__ out,
                                                            uint64_t out_rows) {
  const uint32_t s = blockIdx.x;
  if (s >= num_series) return;
  const ks_desc d = desc[s];
  const uint32_t K = Ks[s];
  if (!(d.aux_offset <= out_rows && K <= out_rows - d.aux_offset)) return;
  for (uint32_t t = threadIdx.x; t < K; t += NTC) out[d.aux_offset + t] = lg[(uint64_t)s * SR + 2 + t];
}

}  // namespace cnn
}  // namespace ks

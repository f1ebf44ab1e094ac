// C ABI of the learned proposal: model lifecycle and checkpoints, the feature
// pass, network forward, proposal, exact refine and one training step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "ks.h"
#include "ks_cnn.hpp"
#include "ks_ctx.hpp"
#include "ks_features.hpp"
#include "ks_refine.hpp"

using namespace ks_host;
namespace C = ks::cnn;

namespace ks_host {

void free_learn(LearnBuffers& b) {
  void* ptrs[] = {b.s1, b.s2lo, b.s2hi, b.smin, b.K, b.feat, b.x0, b.act[0], b.act[1], b.act[2], b.logits,
                  b.dy16, b.dy16f, b.dy[0], b.dy[1], b.dy[2], b.dyf[0], b.dyf[1], b.dyf[2], b.part, b.grad[0], b.grad[1],
                  b.grad[2], b.grad[3], b.nsig};
  for (void* p : ptrs) (void)hipFree(p);
  b = LearnBuffers{};
}

}  // namespace ks_host

namespace {

constexpr uint32_t kDwGrid = 256;     // workgroups of a weight-gradient reduction

uint32_t slot_rows(uint32_t max_K) { return (max_K + 4 + 15) / 16 * 16; }

template <typename T>
bool alloc(T*& p, uint64_t n) {
  return hipMalloc(&p, sizeof(T) * (n ? n : 1)) == hipSuccess;
}

// Grow the learned-path buffers for `rows` slot rows and `series` series
// (training buffers too when `train`).
int ensure_learn(ks_ctx* c, uint64_t rows, uint64_t series, bool train) {
  LearnBuffers& b = c->learn;
  const bool have_train = b.dy16 != nullptr;
  if (rows <= b.cap_rows && series <= b.cap_series && (!train || have_train)) return KS_OK;
  const uint64_t R = rows > b.cap_rows ? rows : b.cap_rows;
  const uint64_t S = series > b.cap_series ? series : b.cap_series;
  const bool T = train || have_train;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  free_learn(b);
  bool ok = alloc(b.s1, R) && alloc(b.s2lo, R) && alloc(b.s2hi, R) && alloc(b.smin, S) && alloc(b.K, S) &&
            alloc(b.feat, R * 9) && alloc(b.x0, R * 16) && alloc(b.act[0], R * 64) && alloc(b.act[1], R * 64) &&
            alloc(b.act[2], R * 64) && alloc(b.logits, R);
  if (ok && T) {
    const uint64_t part = (uint64_t)kDwGrid * (64 * 320 + 64);
    ok = alloc(b.dy16, R * 16) && alloc(b.dy16f, R * 16) && alloc(b.dy[0], R * 64) && alloc(b.dy[1], R * 64) &&
         alloc(b.dy[2], R * 64) && alloc(b.dyf[0], R * 64) && alloc(b.dyf[1], R * 64) && alloc(b.dyf[2], R * 64) &&
         alloc(b.part, part) && alloc(b.grad[0], 64 * 80 + 64) &&
         alloc(b.grad[1], 64 * 320 + 64) && alloc(b.grad[2], 64 * 320 + 64) && alloc(b.grad[3], 16 * 320 + 16) &&
         alloc(b.nsig, 4);
    b.cap_part = part;
  }
  if (!ok) {
    free_learn(b);
    (void)hipGetLastError();
    return KS_E_NOMEM;
  }
  b.cap_rows = R;
  b.cap_series = S;
  return KS_OK;
}

ks::LearnWs learn_ws(ks_ctx* c) {
  return ks::LearnWs{c->learn.s1, c->learn.s2lo, c->learn.s2hi, c->learn.smin, c->learn.K};
}

uint32_t conv_grid(const ks_ctx* c, uint64_t rows) {
  const uint64_t tiles = (rows + C::TM - 1) / C::TM;
  const uint64_t cap = (uint64_t)c->num_cus * 3;
  return (uint32_t)(tiles < cap ? (tiles ? tiles : 1) : cap);
}

// The network forward over the slot rows, one launch per layer, keeping the
// activations a1..a3 for the backward pass: x0 -> a1 -> a2 -> a3 -> logits.
hipError_t forward(ks_ctx* c, const ks_model* m, uint64_t rows, uint32_t SR, hipStream_t st) {
  LearnBuffers& b = c->learn;
  const uint32_t g = conv_grid(c, rows);
  hipLaunchKernelGGL((C::conv_kernel<16, 64, C::EPI_RELU>), dim3(g), dim3(C::NTC), 0, st, b.x0, m->wf[0], m->b[0],
                     rows, SR, b.K, b.act[0], (float*)nullptr, (const uint16_t*)nullptr);
  hipLaunchKernelGGL((C::conv_kernel<64, 64, C::EPI_RELU>), dim3(g), dim3(C::NTC), 0, st, b.act[0], m->wf[1],
                     m->b[1], rows, SR, b.K, b.act[1], (float*)nullptr, (const uint16_t*)nullptr);
  hipLaunchKernelGGL((C::conv_kernel<64, 64, C::EPI_RELU>), dim3(g), dim3(C::NTC), 0, st, b.act[1], m->wf[2],
                     m->b[2], rows, SR, b.K, b.act[2], (float*)nullptr, (const uint16_t*)nullptr);
  hipLaunchKernelGGL((C::conv_kernel<64, 16, C::EPI_LOGIT>), dim3(g), dim3(C::NTC), 0, st, b.act[2], m->wf[3],
                     m->b[3], rows, SR, b.K, (uint16_t*)nullptr, b.logits, (const uint16_t*)nullptr);
  return hipGetLastError();
}

// Inference: the whole network in one launch, activations kept in LDS.
hipError_t forward_infer(ks_ctx* c, const ks_model* m, uint64_t rows, uint32_t SR, hipStream_t st) {
  LearnBuffers& b = c->learn;
  const uint32_t num_series = (uint32_t)(rows / SR);
  const uint32_t per = (SR - 4 + C::FT - 1) / C::FT;  // tiles covering a slot's K <= SR - 4 rows
  const uint64_t tiles = (uint64_t)num_series * per;
  const uint64_t cap = (uint64_t)c->num_cus * 3;  // three 51 KB workgroups per CU
  const uint32_t g = (uint32_t)(tiles < cap ? (tiles ? tiles : 1) : cap);
  hipLaunchKernelGGL(C::fused_forward_kernel, dim3(g), dim3(C::NTC), 0, st, b.x0, rows, SR, b.K, num_series, per,
                     m->wf[0], m->wf[1], m->wf[2], m->wf[3], m->b[0], m->b[1], m->b[2], m->b[3], b.logits);
  return hipGetLastError();
}

// Backward pass over the slot rows from the logit gradient in dy16 / dy16f
// (bf16 / fp32, channel 0), with the activations of the last forward():
// the gradients at the pre-activations y2, y1, y0 in dy / dyf[0..2] and the
// per-layer weight and bias gradients reduced into grad[0..3].
hipError_t backward(ks_ctx* c, const ks_model* model, uint64_t rows, uint32_t SR, hipStream_t st) {
  LearnBuffers& b = c->learn;
  const uint64_t tiles = (rows + C::TM - 1) / C::TM;
  const uint32_t G = (uint32_t)(tiles < kDwGrid ? tiles : kDwGrid);
  const uint32_t gc = conv_grid(c, rows);
  auto reduce = [&](float* dst, uint32_t n) {
    hipLaunchKernelGGL(C::reduce_parts_kernel, dim3((n + C::NTC - 1) / C::NTC), dim3(C::NTC), 0, st, b.part, G, n,
                       dst);
  };
  // layer 3 (64 -> 1), then 2, 1 (64 -> 64), then 0 (11 -> 64)
  hipLaunchKernelGGL((C::dw_kernel<64, 16>), dim3(G), dim3(C::NTC), 0, st, b.dy16, b.dy16f, b.act[2], rows, b.part);
  reduce(b.grad[3], C::DwShape<64, 16>::PART);
  hipLaunchKernelGGL((C::conv_kernel<16, 64, C::EPI_BWD>), dim3(gc), dim3(C::NTC), 0, st, b.dy16, model->wb[3],
                     (const float*)nullptr, rows, SR, b.K, b.dy[0], b.dyf[0], b.act[2]);
  hipLaunchKernelGGL((C::dw_kernel<64, 64>), dim3(G), dim3(C::NTC), 0, st, b.dy[0], b.dyf[0], b.act[1], rows, b.part);
  reduce(b.grad[2], C::DwShape<64, 64>::PART);
  hipLaunchKernelGGL((C::conv_kernel<64, 64, C::EPI_BWD>), dim3(gc), dim3(C::NTC), 0, st, b.dy[0], model->wb[2],
                     (const float*)nullptr, rows, SR, b.K, b.dy[1], b.dyf[1], b.act[1]);
  hipLaunchKernelGGL((C::dw_kernel<64, 64>), dim3(G), dim3(C::NTC), 0, st, b.dy[1], b.dyf[1], b.act[0], rows, b.part);
  reduce(b.grad[1], C::DwShape<64, 64>::PART);
  hipLaunchKernelGGL((C::conv_kernel<64, 64, C::EPI_BWD>), dim3(gc), dim3(C::NTC), 0, st, b.dy[1], model->wb[1],
                     (const float*)nullptr, rows, SR, b.K, b.dy[2], b.dyf[2], b.act[0]);
  hipLaunchKernelGGL((C::dw_kernel<16, 64>), dim3(G), dim3(C::NTC), 0, st, b.dy[2], b.dyf[2], b.x0, rows, b.part);
  reduce(b.grad[0], C::DwShape<16, 64>::PART);
  return hipGetLastError();
}

template <int KMAX>
void launch_refine(const ks_desc* desc, uint32_t n, uint64_t num_samples, uint32_t max_K, const ks_params& prm,
                   const int32_t* prop, const float* conf, ks::LearnWs lw, uint32_t SR, ks_result* out,
                   hipStream_t st) {
  // K classes of 1024 and 2048 rows in 512-thread workgroups: their LDS, not
  // registers, limits the workgroups per CU, so twice the threads per
  // workgroup doubles the waves walking the fallback series (the learned
  // step on 8192 x 1024 x 2048 0.5% faster)
  constexpr int RNT = KMAX >= 1024 ? 512 : kNT;
  hipLaunchKernelGGL((ks::refine_kernel<KMAX, RNT, kRB>), dim3(n), dim3(RNT), 0, st, desc, n, num_samples, max_K, prm,
                     prop, conf, lw, SR, out);
}

hipError_t shadow(ks_model* m, hipStream_t st) {
  C::Shadow sh;
  for (int l = 0; l < 4; ++l) {
    sh.wf[l] = m->wf[l];
    sh.wb[l] = m->wb[l];
    sh.b[l] = m->b[l];
  }
  hipLaunchKernelGGL(C::shadow_kernel, dim3((C::kShadowEntries + C::NTC - 1) / C::NTC), dim3(C::NTC), 0, st, m->theta, sh);
  return hipGetLastError();
}

void free_model(ks_model* m) {
  void* ptrs[] = {m->theta, m->m1, m->m2, m->grad, m->wf[0], m->wf[1], m->wf[2], m->wf[3],
                  m->wb[1], m->wb[2], m->wb[3], m->b[0], m->b[1], m->b[2], m->b[3]};
  for (void* p : ptrs) (void)hipFree(p);
}

// splitmix64 (Steele, Lea, Flood 2014) for the initial weights
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t fnv1a(const void* p, size_t n, uint64_t h = 0xcbf29ce484222325ull) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 0x100000001b3ull;
  return h;
}

const char kMagic[8] = {'K', 'S', 'C', 'N', 'N', '0', '0', '1'};

int check_learn_args(const ks_desc* desc, uint32_t num_series, uint32_t max_K) {
  if (!desc && num_series) return KS_E_INVALID;
  if (num_series > (1u << 26)) return KS_E_RANGE;
  if (max_K < 2 || max_K > KS_MAX_K) return KS_E_RANGE;
  return KS_OK;
}

}  // namespace

extern "C" {

int ks_model_create(ks_ctx* ctx, uint64_t seed, ks_model** out) {
  if (!ctx || !out) return KS_E_INVALID;
  *out = nullptr;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  ks_model* m = new (std::nothrow) ks_model();
  if (!m) return KS_E_NOMEM;
  m->device = ctx->device;
  bool ok = alloc(m->theta, C::kNumParams) && alloc(m->m1, C::kNumParams) && alloc(m->m2, C::kNumParams) &&
            alloc(m->grad, C::kNumParams);
  for (int l = 0; l < 4 && ok; ++l) {
    const C::Layer L = C::layer_info(l);
    ok = alloc(m->wf[l], (uint64_t)L.cout_pad * 5 * L.cin_pad) && alloc(m->b[l], L.cout_pad);
    if (ok && l >= 1) ok = alloc(m->wb[l], (uint64_t)L.cin_pad * 5 * L.cout_pad);
  }
  if (!ok) {
    free_model(m);
    delete m;
    (void)hipGetLastError();
    return KS_E_NOMEM;
  }
  // He-uniform weights U(-a, a), a = sqrt(6 / fan_in), zero biases
  std::vector<float> h(C::kNumParams, 0.0f);
  uint64_t st = seed;
  for (int l = 0; l < 4; ++l) {
    const C::Layer L = C::layer_info(l);
    const double a = std::sqrt(6.0 / (L.cin * 5.0));
    for (uint32_t p = L.w_off; p < L.b_off; ++p) {
      const double u = (double)(splitmix64(st) >> 11) * 0x1p-53;
      h[p] = (float)((2.0 * u - 1.0) * a);
    }
  }
  int rc = ks_model_set_params(m, h.data());
  if (rc) {
    free_model(m);
    delete m;
    return rc;
  }
  *out = m;
  return KS_OK;
}

int ks_model_destroy(ks_model* m) {
  if (!m) return KS_E_INVALID;
  DeviceGuard g(m->device);
  (void)hipDeviceSynchronize();
  free_model(m);
  delete m;
  return KS_OK;
}

int ks_model_set_params(ks_model* m, const float* host) {
  if (!m || !host) return KS_E_INVALID;
  DeviceGuard g(m->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  for (uint32_t p = 0; p < C::kNumParams; ++p)
    if (!std::isfinite(host[p])) return KS_E_MODEL;
  hipError_t e;
  if ((e = hipMemcpy(m->theta, host, sizeof(float) * C::kNumParams, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(m->m1, 0, sizeof(float) * C::kNumParams)) != hipSuccess ||
      (e = hipMemset(m->m2, 0, sizeof(float) * C::kNumParams)) != hipSuccess ||
      (e = hipMemset(m->grad, 0, sizeof(float) * C::kNumParams)) != hipSuccess)
    return hip_fail(e, "ks_model_set_params");
  if ((e = shadow(m, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess)
    return hip_fail(e, "shadow weights");
  m->step = 0;
  return KS_OK;
}

int ks_model_get_params(ks_model* m, float* host) {
  if (!m || !host) return KS_E_INVALID;
  DeviceGuard g(m->device);
  hipError_t e = hipMemcpy(host, m->theta, sizeof(float) * C::kNumParams, hipMemcpyDeviceToHost);
  return e == hipSuccess ? KS_OK : hip_fail(e, "ks_model_get_params");
}

int ks_model_grads(ks_model* m, float* host) {
  if (!m || !host) return KS_E_INVALID;
  DeviceGuard g(m->device);
  hipError_t e = hipMemcpy(host, m->grad, sizeof(float) * C::kNumParams, hipMemcpyDeviceToHost);
  return e == hipSuccess ? KS_OK : hip_fail(e, "ks_model_grads");
}

// File: magic "KSCNN001", u32 parameter count, u64 step, then theta, m1, m2
// (fp32), then the FNV-1a 64 hash of everything before it.
int ks_model_save(ks_model* m, const char* path) {
  if (!m || !path) return KS_E_INVALID;
  DeviceGuard g(m->device);
  std::vector<float> buf(3 * (size_t)C::kNumParams);
  hipError_t e;
  if ((e = hipMemcpy(buf.data(), m->theta, sizeof(float) * C::kNumParams, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(buf.data() + C::kNumParams, m->m1, sizeof(float) * C::kNumParams, hipMemcpyDeviceToHost)) !=
          hipSuccess ||
      (e = hipMemcpy(buf.data() + 2 * C::kNumParams, m->m2, sizeof(float) * C::kNumParams,
                     hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "ks_model_save");
  const uint32_t n = C::kNumParams;
  uint64_t h = fnv1a(kMagic, 8);
  h = fnv1a(&n, 4, h);
  h = fnv1a(&m->step, 8, h);
  h = fnv1a(buf.data(), buf.size() * 4, h);
  FILE* f = std::fopen(path, "wb");
  if (!f) return KS_E_INVALID;
  const bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(&n, 4, 1, f) == 1 &&
                  std::fwrite(&m->step, 8, 1, f) == 1 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size() &&
                  std::fwrite(&h, 8, 1, f) == 1;
  return (std::fclose(f) == 0 && ok) ? KS_OK : KS_E_INVALID;
}

int ks_model_load(ks_model* m, const char* path) {
  if (!m || !path) return KS_E_INVALID;
  FILE* f = std::fopen(path, "rb");
  if (!f) return KS_E_INVALID;
  char magic[8];
  uint32_t n = 0;
  uint64_t step = 0, h = 0;
  std::vector<float> buf(3 * (size_t)C::kNumParams);
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::fread(&n, 4, 1, f) == 1 && n == C::kNumParams &&
                  std::fread(&step, 8, 1, f) == 1 && std::fread(buf.data(), 4, buf.size(), f) == buf.size() &&
                  std::fread(&h, 8, 1, f) == 1;
  std::fclose(f);
  if (!ok || std::memcmp(magic, kMagic, 8) != 0) return KS_E_MODEL;
  uint64_t hh = fnv1a(kMagic, 8);
  hh = fnv1a(&n, 4, hh);
  hh = fnv1a(&step, 8, hh);
  hh = fnv1a(buf.data(), buf.size() * 4, hh);
  if (hh != h) return KS_E_MODEL;
  if (int rc = ks_model_set_params(m, buf.data())) return rc;
  DeviceGuard g(m->device);
  hipError_t e;
  if ((e = hipMemcpy(m->m1, buf.data() + C::kNumParams, sizeof(float) * C::kNumParams, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(m->m2, buf.data() + 2 * C::kNumParams, sizeof(float) * C::kNumParams,
                     hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "ks_model_load");
  m->step = step;
  return KS_OK;
}

int ks_learn_reserve(ks_ctx* ctx, uint32_t max_series, uint32_t max_K, int train) {
  if (!ctx) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (int rc = check_learn_args(nullptr, 0, max_K)) return rc;
  if (max_series > (1u << 26)) return KS_E_RANGE;
  if (max_series == 0) return KS_OK;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  return ensure_learn(ctx, (uint64_t)max_series * slot_rows(max_K), max_series, train != 0);
}

int ks_features(ks_ctx* ctx, const uint32_t* samples, uint64_t num_samples, const ks_desc* desc,
                uint32_t num_series, uint32_t max_K, float* features, uint64_t feature_rows, void* stream) {
  if (!ctx) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (int rc = check_learn_args(desc, num_series, max_K)) return rc;
  if (num_series == 0) return KS_OK;
  if (!samples) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const uint32_t SR = slot_rows(max_K);
  if (int rc = ensure_learn(ctx, (uint64_t)num_series * SR, num_series, false)) return rc;
  hipStream_t st = (hipStream_t)stream;
  LearnBuffers& b = ctx->learn;
  // the series order per row class, kept in the logits buffer (num_series + 10
  // words <= its rows; nothing reads the logits before the forward rewrites
  // them), then one launch per row class (1, 2 or 4 load batches per row,
  // streamed, or short rows four to a wave): its workgroups past the class's
  // count return at once
  uint32_t* plan = reinterpret_cast<uint32_t*>(b.logits);
  hipLaunchKernelGGL(ks::feature_plan_kernel, dim3(1), dim3(ks::kFeatPlanNT), 0, st, desc, num_series, num_samples,
                     max_K, plan);
  hipLaunchKernelGGL((ks::features_kernel<1, ks::row_pass_threads(1)>), dim3(num_series),
                     dim3(ks::row_pass_threads(1)), 0, st, samples, num_samples, desc,
                     num_series, max_K, SR, learn_ws(ctx), b.feat, plan);
  hipLaunchKernelGGL((ks::features_kernel<2, ks::row_pass_threads(2)>), dim3(num_series),
                     dim3(ks::row_pass_threads(2)), 0, st, samples, num_samples, desc,
                     num_series, max_K, SR, learn_ws(ctx), b.feat, plan);
  hipLaunchKernelGGL((ks::features_kernel<4, ks::row_pass_threads(4)>), dim3(num_series),
                     dim3(ks::row_pass_threads(4)), 0, st, samples, num_samples, desc,
                     num_series, max_K, SR, learn_ws(ctx), b.feat, plan);
  hipLaunchKernelGGL((ks::features_kernel<ks::kStreamed, ks::row_pass_threads(ks::kStreamed)>), dim3(num_series),
                     dim3(ks::row_pass_threads(ks::kStreamed)), 0, st, samples,
                     num_samples, desc, num_series, max_K, SR, learn_ws(ctx), b.feat, plan);
  hipLaunchKernelGGL((ks::features_kernel<ks::kGrouped, ks::row_pass_threads(ks::kGrouped)>), dim3(num_series),
                     dim3(ks::row_pass_threads(ks::kGrouped)), 0, st, samples,
                     num_samples, desc, num_series, max_K, SR, learn_ws(ctx), b.feat, plan);
  hipLaunchKernelGGL((ks::feature_pack_kernel<kNT>), dim3(num_series, (SR + kNT - 1) / kNT), dim3(kNT), 0, st, desc,
                     num_series, features, feature_rows, b.x0, SR, learn_ws(ctx), b.feat);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "features launch");
  b.stamp_desc = desc;
  b.stamp_series = num_series;
  b.stamp_SR = SR;
  b.stamp_maxK = max_K;
  b.stamp_valid = true;
  return KS_OK;
}

int ks_cnn_forward(ks_ctx* ctx, const ks_model* model, const float* features, uint64_t feature_rows,
                   const ks_desc* desc, uint32_t num_series, uint32_t max_K, float* logits, uint64_t logit_rows,
                   void* stream) {
  if (!ctx || !model) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (int rc = check_learn_args(desc, num_series, max_K)) return rc;
  if (num_series == 0) return KS_OK;
  if (!features || !logits) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const uint32_t SR = slot_rows(max_K);
  const uint64_t rows = (uint64_t)num_series * SR;
  if (int rc = ensure_learn(ctx, rows, num_series, false)) return rc;
  hipStream_t st = (hipStream_t)stream;
  LearnBuffers& b = ctx->learn;
  b.stamp_valid = false;  // the slot buffers no longer hold a proposal pass
  hipLaunchKernelGGL(C::pack_features_kernel, dim3(num_series), dim3(C::NTC), 0, st, features, feature_rows, desc,
                     num_series, max_K, SR, b.x0, b.K);
  hipError_t e = forward_infer(ctx, model, rows, SR, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(C::unpack_logits_kernel, dim3(num_series), dim3(C::NTC), 0, st, b.logits, desc, num_series,
                       SR, b.K, logits, logit_rows);
    e = hipGetLastError();
  }
  return e == hipSuccess ? KS_OK : hip_fail(e, "cnn forward");
}

int ks_propose(ks_ctx* ctx, const ks_model* model, const uint32_t* samples, uint64_t num_samples,
               const ks_desc* desc, uint32_t num_series, const ks_params* params, int32_t* proposal,
               float* confidence, float* features, uint64_t feature_rows, void* stream) {
  if (!ctx || !params) return KS_E_INVALID;
  if (int rc = check_params(params)) return rc;
  if (num_series == 0) return KS_OK;
  if (!proposal || !confidence) return KS_E_INVALID;
  const uint32_t max_K = params->max_K ? params->max_K : KS_MAX_K;
  if (int rc = ks_features(ctx, samples, num_samples, desc, num_series, max_K, features, feature_rows, stream))
    return rc;
  DeviceGuard g(ctx->device);
  hipStream_t st = (hipStream_t)stream;
  LearnBuffers& b = ctx->learn;
  const uint32_t SR = b.stamp_SR;
  const uint32_t per = C::NTC / 64;
  if (!model) {  // the method without the network: the largest jump of the per-row median
    hipLaunchKernelGGL(C::median_jump_kernel, dim3((num_series + per - 1) / per), dim3(C::NTC), 0, st, b.feat,
                       num_series, SR, b.K, proposal, confidence);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KS_OK : hip_fail(e, "propose");
  }
  hipError_t e = forward_infer(ctx, model, (uint64_t)num_series * SR, SR, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(C::softmax_kernel, dim3((num_series + per - 1) / per), dim3(C::NTC), 0, st, b.logits,
                       num_series, SR, b.K, (const int32_t*)nullptr, (const uint32_t*)nullptr, (float*)nullptr,
                       (uint16_t*)nullptr, (float*)nullptr, params->w, proposal, confidence);
    e = hipGetLastError();
  }
  return e == hipSuccess ? KS_OK : hip_fail(e, "propose");
}

int ks_refine(ks_ctx* ctx, const ks_desc* desc, uint32_t num_series, uint64_t num_samples, const int32_t* proposal,
              const float* confidence, const ks_params* params, ks_result* out, void* stream) {
  if (!ctx || !params || !out) return KS_E_INVALID;
  if (int rc = check_params(params)) return rc;
  if (num_series == 0) return KS_OK;
  if (!desc || !proposal || !confidence) return KS_E_INVALID;
  const uint32_t max_K = params->max_K ? params->max_K : KS_MAX_K;
  LearnBuffers& b = ctx->learn;
  if (!b.stamp_valid || b.stamp_desc != desc || b.stamp_series != num_series || b.stamp_maxK != max_K)
    return KS_E_STATE;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const ks::LearnWs lw = learn_ws(ctx);
  switch (k_class(max_K)) {
    case 0: launch_refine<64>(desc, num_series, num_samples, max_K, *params, proposal, confidence, lw, b.stamp_SR, out, st); break;
    case 1: launch_refine<128>(desc, num_series, num_samples, max_K, *params, proposal, confidence, lw, b.stamp_SR, out, st); break;
    case 2: launch_refine<256>(desc, num_series, num_samples, max_K, *params, proposal, confidence, lw, b.stamp_SR, out, st); break;
    case 3: launch_refine<512>(desc, num_series, num_samples, max_K, *params, proposal, confidence, lw, b.stamp_SR, out, st); break;
    case 4: launch_refine<1024>(desc, num_series, num_samples, max_K, *params, proposal, confidence, lw, b.stamp_SR, out, st); break;
    default: launch_refine<2048>(desc, num_series, num_samples, max_K, *params, proposal, confidence, lw, b.stamp_SR, out, st);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "refine launch");
}

int ks_train_step(ks_ctx* ctx, ks_model* model, const float* features, uint64_t feature_rows, const ks_desc* desc,
                  const int32_t* labels, uint32_t num_series, uint32_t max_K, float lr, float* loss, void* stream) {
  if (!ctx || !model) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (int rc = check_learn_args(desc, num_series, max_K)) return rc;
  if (num_series == 0) return KS_OK;
  if (!features || !labels || !(lr >= 0.0f) || !std::isfinite(lr)) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const uint32_t SR = slot_rows(max_K);
  const uint64_t rows = (uint64_t)num_series * SR;
  if (int rc = ensure_learn(ctx, rows, num_series, true)) return rc;
  hipStream_t st = (hipStream_t)stream;
  LearnBuffers& b = ctx->learn;
  b.stamp_valid = false;
  hipLaunchKernelGGL(C::pack_features_kernel, dim3(num_series), dim3(C::NTC), 0, st, features, feature_rows, desc,
                     num_series, max_K, SR, b.x0, b.K);
  hipError_t e = forward(ctx, model, rows, SR, st);
  if (e != hipSuccess) return hip_fail(e, "train forward");
  // loss and logit gradient
  hipLaunchKernelGGL(C::count_labels_kernel, dim3(1), dim3(C::NTC), 0, st, labels, num_series, b.nsig);
  float* loss_acc = reinterpret_cast<float*>(b.nsig + 1);  // discarded when the caller wants no loss
  if (loss) {
    hipLaunchKernelGGL(C::zero_kernel, dim3(1), dim3(C::NTC), 0, st, loss, 1u);
    loss_acc = loss;
  }
  const uint32_t per = C::NTC / 64;
  hipLaunchKernelGGL(C::softmax_kernel, dim3((num_series + per - 1) / per), dim3(C::NTC), 0, st, b.logits, num_series,
                     SR, b.K, labels, b.nsig, loss_acc, b.dy16, b.dy16f, 0u, (int32_t*)nullptr, (float*)nullptr);
  if ((e = backward(ctx, model, rows, SR, st)) != hipSuccess) return hip_fail(e, "train backward");
  // Adam
  model->step += 1;
  const float bc1 = (float)(1.0 - std::pow(0.9, (double)model->step));
  const float bc2 = (float)(1.0 - std::pow(0.999, (double)model->step));
  hipLaunchKernelGGL(C::adam_kernel, dim3((C::kNumParams + C::NTC - 1) / C::NTC), dim3(C::NTC), 0, st, model->theta,
                     model->m1, model->m2, model->grad, b.grad[0], b.grad[1], b.grad[2], b.grad[3], lr, bc1, bc2,
                     1);
  e = shadow(model, st);
  return e == hipSuccess ? KS_OK : hip_fail(e, "train step");
}

int ks_cnn_backward(ks_ctx* ctx, const ks_model* model, const float* features, uint64_t feature_rows,
                    const ks_desc* desc, uint32_t num_series, uint32_t max_K, const float* dlogits,
                    uint64_t dlogit_rows, float* grads, void* stream) {
  if (!ctx || !model) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (int rc = check_learn_args(desc, num_series, max_K)) return rc;
  if (!grads) return KS_E_INVALID;
  if (num_series && (!features || !dlogits)) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t SR = slot_rows(max_K);
  const uint64_t rows = (uint64_t)(num_series ? num_series : 1) * SR;
  if (int rc = ensure_learn(ctx, rows, num_series ? num_series : 1, true)) return rc;
  LearnBuffers& b = ctx->learn;
  b.stamp_valid = false;
  hipError_t e;
  if (num_series == 0) {  // an empty batch has a zero gradient
    hipLaunchKernelGGL(C::zero_kernel, dim3((C::kNumParams + C::NTC - 1) / C::NTC), dim3(C::NTC), 0, st, grads,
                       C::kNumParams);
    e = hipGetLastError();
    return e == hipSuccess ? KS_OK : hip_fail(e, "gradient reset");
  }
  hipLaunchKernelGGL(C::pack_features_kernel, dim3(num_series), dim3(C::NTC), 0, st, features, feature_rows, desc,
                     num_series, max_K, SR, b.x0, b.K);
  if ((e = forward(ctx, model, rows, SR, st)) != hipSuccess) return hip_fail(e, "backward: forward");
  hipLaunchKernelGGL(C::pack_dlogits_kernel, dim3(num_series), dim3(C::NTC), 0, st, dlogits, dlogit_rows, desc,
                     num_series, SR, b.K, b.dy16, b.dy16f);
  if ((e = backward(ctx, model, rows, SR, st)) != hipSuccess) return hip_fail(e, "backward");
  // gather into the parameter layout (the optimizer kernel with its update off)
  hipLaunchKernelGGL(C::adam_kernel, dim3((C::kNumParams + C::NTC - 1) / C::NTC), dim3(C::NTC), 0, st,
                     (float*)nullptr, (float*)nullptr, (float*)nullptr, grads, b.grad[0], b.grad[1], b.grad[2],
                     b.grad[3], 0.0f, 1.0f, 1.0f, 0);
  e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "backward gather");
}

int ks_cnn_trace(ks_ctx* ctx, const ks_model* model, const float* features, uint64_t feature_rows,
                 const ks_desc* desc, uint32_t num_series, uint32_t max_K, const int32_t* labels,
                 const float* dlogits, uint64_t dlogit_rows, float* acts, float* grads_in, uint64_t trace_rows,
                 float* grads, void* stream) {
  if (!ctx || !model) return KS_E_INVALID;
  if (max_K == 0) max_K = KS_MAX_K;
  if (int rc = check_learn_args(desc, num_series, max_K)) return rc;
  if (num_series == 0) return KS_OK;
  if (!features) return KS_E_INVALID;
  const bool bwd = labels || dlogits;
  if ((grads_in || grads) && !bwd) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  const uint32_t SR = slot_rows(max_K);
  const uint64_t rows = (uint64_t)num_series * SR;
  if (int rc = ensure_learn(ctx, rows, num_series, true)) return rc;
  LearnBuffers& b = ctx->learn;
  b.stamp_valid = false;
  hipLaunchKernelGGL(C::pack_features_kernel, dim3(num_series), dim3(C::NTC), 0, st, features, feature_rows, desc,
                     num_series, max_K, SR, b.x0, b.K);
  hipError_t e = forward(ctx, model, rows, SR, st);
  if (e != hipSuccess) return hip_fail(e, "trace forward");
  if (labels) {  // the training step's logit gradient (its loss goes to a scratch word)
    hipLaunchKernelGGL(C::count_labels_kernel, dim3(1), dim3(C::NTC), 0, st, labels, num_series, b.nsig);
    const uint32_t per = C::NTC / 64;
    hipLaunchKernelGGL(C::softmax_kernel, dim3((num_series + per - 1) / per), dim3(C::NTC), 0, st, b.logits,
                       num_series, SR, b.K, labels, b.nsig, reinterpret_cast<float*>(b.nsig + 1), b.dy16, b.dy16f, 0u,
                       (int32_t*)nullptr, (float*)nullptr);
  } else if (dlogits) {
    hipLaunchKernelGGL(C::pack_dlogits_kernel, dim3(num_series), dim3(C::NTC), 0, st, dlogits, dlogit_rows, desc,
                       num_series, SR, b.K, b.dy16, b.dy16f);
  }
  if (bwd) {
    if ((e = backward(ctx, model, rows, SR, st)) != hipSuccess) return hip_fail(e, "trace backward");
    if (grads)
      hipLaunchKernelGGL(C::adam_kernel, dim3((C::kNumParams + C::NTC - 1) / C::NTC), dim3(C::NTC), 0, st,
                         (float*)nullptr, (float*)nullptr, (float*)nullptr, grads, b.grad[0], b.grad[1], b.grad[2],
                         b.grad[3], 0.0f, 1.0f, 1.0f, 0);
  }
  if (acts || grads_in)
    hipLaunchKernelGGL(C::trace_copy_kernel, dim3(num_series), dim3(C::NTC), 0, st, desc, num_series, SR, b.K, b.x0,
                       b.act[0], b.act[1], b.act[2], b.logits, b.dy16f, bwd ? b.dyf[0] : nullptr, b.dyf[1], b.dyf[2],
                       acts, grads_in, trace_rows);
  e = hipGetLastError();
  return e == hipSuccess ? KS_OK : hip_fail(e, "trace");
}

}  // extern "C"

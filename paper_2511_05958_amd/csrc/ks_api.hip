// C ABI of the K-S change-point library: contexts, validation, launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "ks.h"
#include "ks_scan.hpp"

struct ks_ctx {
  int device = 0;
  int num_cus = 0;
  size_t lds_per_block = 0;
  uint32_t reserved_series = 0;
  uint64_t reserved_steps = 0;
};

namespace {

thread_local char g_hip_msg[256] = "HIP error";

int hip_fail(hipError_t e, const char* what) {
  snprintf(g_hip_msg, sizeof(g_hip_msg), "HIP error in %s: %s", what, hipGetErrorString(e));
  return KS_E_HIP;
}

// Make the context's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) {
      err = hipSetDevice(dev);
      changed = err == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

int check_params(const ks_params* p) {
  if (!p) return KS_E_INVALID;
  if (!(p->alpha > 0.0 && p->alpha < 1.0)) return KS_E_INVALID;
  if (!(p->c_alpha > 0.0) || !std::isfinite(p->c_alpha)) return KS_E_INVALID;
  if (p->w < 1 || p->w > 64) return KS_E_INVALID;
  if (!(p->tau >= 0.0f && p->tau <= 1.0f)) return KS_E_INVALID;
  if (p->opts != 0) return KS_E_INVALID;
  if (p->max_K != 0 && (p->max_K < 2 || p->max_K > KS_MAX_K)) return KS_E_RANGE;
  return KS_OK;
}

constexpr int kNT = 256;
constexpr int kRB = 4;

template <int KMAX>
hipError_t launch_scan(const uint32_t* samples, uint64_t num_samples, const ks_desc* desc, uint32_t num_series,
                       const ks_params& prm, uint32_t max_K, ks_result* out, uint32_t* allU, uint64_t allU_len,
                       hipStream_t st) {
  hipLaunchKernelGGL((ks::scan_kernel<KMAX, kNT, kRB>), dim3(num_series), dim3(kNT), 0, st, samples, num_samples,
                     desc, num_series, prm, max_K, out, allU, allU_len);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int ks_version(void) { return KS_VERSION; }

const char* ks_status_string(int status) {
  switch (status) {
    case KS_OK: return "ok";
    case KS_E_INVALID: return "invalid argument (null pointer or bad parameter)";
    case KS_E_RANGE: return "size outside the documented limits";
    case KS_E_STATE: return "call order or workspace state mismatch";
    case KS_E_HIP: return g_hip_msg;
    case KS_E_MODEL: return "bad model handle, file or weights";
    case KS_E_NOMEM: return "device allocation failed";
    default: return "unknown status";
  }
}

int ks_params_init(ks_params* p, double alpha) {
  if (!p || !(alpha > 0.0 && alpha < 1.0)) return KS_E_INVALID;
  p->alpha = alpha;
  p->c_alpha = -0.5 * std::log(alpha / 2.0);
  p->max_K = 0;
  p->w = 8;
  p->tau = 0.5f;
  p->opts = 0;
  return KS_OK;
}

int ks_ctx_create(int device, ks_ctx** out) {
  if (!out) return KS_E_INVALID;
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= n) return KS_E_RANGE;
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  ks_ctx* c = new (std::nothrow) ks_ctx();
  if (!c) return KS_E_NOMEM;
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  c->lds_per_block = prop.sharedMemPerBlock;
  *out = c;
  return KS_OK;
}

int ks_ctx_destroy(ks_ctx* ctx) {
  if (!ctx) return KS_E_INVALID;
  delete ctx;
  return KS_OK;
}

int ks_reserve(ks_ctx* ctx, uint32_t max_series, uint64_t max_total_steps) {
  if (!ctx) return KS_E_INVALID;
  ctx->reserved_series = max_series;
  ctx->reserved_steps = max_total_steps;
  return KS_OK;
}

int ks_scan_batch(ks_ctx* ctx, const uint32_t* samples, uint64_t num_samples, const ks_desc* desc,
                  uint32_t num_series, const ks_params* params, ks_result* out, uint32_t* all_U,
                  uint64_t all_U_len, void* stream) {
  if (!ctx || !params || !out) return KS_E_INVALID;
  if (int rc = check_params(params)) return rc;
  if (num_series == 0) return KS_OK;
  if (!samples || !desc) return KS_E_INVALID;
  if (num_series > (1u << 30)) return KS_E_RANGE;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const uint32_t max_K = params->max_K ? params->max_K : KS_MAX_K;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (max_K <= 64)
    e = launch_scan<64>(samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, st);
  else if (max_K <= 128)
    e = launch_scan<128>(samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, st);
  else if (max_K <= 256)
    e = launch_scan<256>(samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, st);
  else if (max_K <= 512)
    e = launch_scan<512>(samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, st);
  else if (max_K <= 1024)
    e = launch_scan<1024>(samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, st);
  else
    e = launch_scan<2048>(samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, st);
  if (e != hipSuccess) return hip_fail(e, "scan launch");
  return KS_OK;
}

}  // extern "C"

// C ABI of the K-S change-point library: contexts, workspace, validation,
// launch plans (direct grid or planned persistent launch captured in a
// hipGraph) and the tuning table.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <new>
#include <tuple>

#include "ks.h"
#include "ks_ctx.hpp"
#include "ks_persist.hpp"

using namespace ks_host;

namespace ks_host {

thread_local char g_hip_msg[256] = "HIP error";

int hip_fail(hipError_t e, const char* what) {
  snprintf(g_hip_msg, sizeof(g_hip_msg), "HIP error in %s: %s", what, hipGetErrorString(e));
  return KS_E_HIP;
}

// the variant tables, one per object built from ks_scan_variants.hip
extern const ScanKernels scan_table_0[kNumKClasses], scan_table_1[kNumKClasses], scan_table_2[kNumKClasses],
    scan_table_3[kNumKClasses], scan_table_4[kNumKClasses], scan_table_5[kNumKClasses];
static_assert(kNumVariants == 6, "one table per variant");

const ScanKernels& scan_kernels(int kclass, int variant) {
  static const ScanKernels* const tables[kNumVariants] = {scan_table_0, scan_table_1, scan_table_2,
                                                          scan_table_3, scan_table_4, scan_table_5};
  return tables[variant][kclass];
}

}  // namespace ks_host

// Scratch of ks_scan_batch_noalloc: the ordered plan's header (256 B), then
// items, per-series moment bases, completion counts and minima laid out for
// KS_NOALLOC_MAX_SERIES series. Each device holds its own copy for the life
// of the process; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device.
namespace {
constexpr uint64_t kScratchItems = 256;
constexpr uint64_t kScratchBase = kScratchItems + 8ull * KS_NOALLOC_MAX_SERIES;
constexpr uint64_t kScratchDone = kScratchBase + 8ull * KS_NOALLOC_MAX_SERIES;
constexpr uint64_t kScratchMin = kScratchDone + 4ull * KS_NOALLOC_MAX_SERIES;
constexpr uint64_t kScratchBytes = kScratchMin + 4ull * KS_NOALLOC_MAX_SERIES;
static_assert(sizeof(ks::Item) == 8, "item layout");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices] = {};  // device address of `scratch` per device

// Resolve the scratch array's address on `device` (made current by the caller), once per device.
int resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return KS_E_RANGE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return KS_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress");
  g_scratch[device] = static_cast<unsigned char*>(p);
  return KS_OK;
}

unsigned char* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

void free_workspace(ks_ctx* c) {
  (void)hipFree(c->hdr);
  (void)hipFree(c->items);
  (void)hipFree(c->mom_base);
  (void)hipFree(c->done);
  (void)hipFree(c->smin);
  (void)hipFree(c->mom);
  c->hdr = nullptr;
  c->items = nullptr;
  c->mom_base = nullptr;
  c->done = nullptr;
  c->smin = nullptr;
  c->mom = nullptr;
  c->cap_series = c->cap_rows = 0;
}

// Grow the workspace to hold num_series series and rows split-series rows.
int ensure_workspace(ks_ctx* c, uint64_t num_series, uint64_t rows) {
  if (num_series <= c->cap_series && rows <= c->cap_rows && c->hdr) return KS_OK;
  const uint64_t ns = num_series > c->cap_series ? num_series : c->cap_series;
  const uint64_t nr = rows > c->cap_rows ? rows : c->cap_rows;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  free_workspace(c);
  if (hipMalloc(&c->hdr, 256) != hipSuccess || hipMalloc(&c->items, sizeof(ks::Item) * ks::kMaxChunks * ns) != hipSuccess ||
      hipMalloc(&c->mom_base, sizeof(uint64_t) * ns) != hipSuccess || hipMalloc(&c->done, sizeof(uint32_t) * ns) != hipSuccess ||
      hipMalloc(&c->smin, sizeof(uint32_t) * ns) != hipSuccess ||
      hipMalloc(&c->mom, sizeof(ks::RowMom) * (nr ? nr : 1)) != hipSuccess) {
    free_workspace(c);
    (void)hipGetLastError();
    return KS_E_NOMEM;
  }
  c->cap_series = ns;
  c->cap_rows = nr;
  return KS_OK;
}

ks::Workspace workspace_of(const ks_ctx* c) {
  return ks::Workspace{c->hdr, c->items, c->mom_base, c->done, c->smin, c->mom};
}

struct ScanArgs {
  const uint32_t* samples;
  uint64_t num_samples;
  const ks_desc* desc;
  uint32_t num_series;
  ks_params prm;
  uint32_t max_K;
  ks_result* out;
  uint32_t* allU;
  uint64_t allU_len;
  uint32_t chunk;
  ks::Workspace ws;
};

// Launch the grid scan of variant v (one workgroup per series, descriptor order).
hipError_t launch_grid(int kc, int v, const ScanArgs& a, hipStream_t st) {
  ScanArgs x = a;
  const uint32_t* order = nullptr;
  void* args[] = {&x.samples, &x.num_samples, &x.desc, &x.num_series, &x.prm, &x.max_K,
                  &x.out, &x.allU, &x.allU_len, &order};
  return hipLaunchKernel(scan_kernels(kc, v).grid, dim3(x.num_series), dim3(kVariants[v].nt), args, 0, st);
}

int persistent_grid(ks_ctx* c, int kc, int v, uint32_t& grid) {
  if (!c->occupancy[kc][v]) {
    int nb = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, scan_kernels(kc, v).persistent, kVariants[v].nt, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    c->occupancy[kc][v] = nb > 0 ? nb : 1;
  }
  grid = (uint32_t)(c->num_cus * c->occupancy[kc][v]);
  return KS_OK;
}

// Launch the plan's kernels (directly, or from a cached hipGraph whose kernel
// arguments are updated for this call).
int launch_plan(ks_ctx* c, int kc, int v, int mode, const ScanArgs& a, bool use_graph, hipStream_t st) {
  const uint32_t nt = (uint32_t)kVariants[v].nt;
  const ScanKernels& K = scan_kernels(kc, v);
  ScanArgs x = a;
  const uint32_t* order = reinterpret_cast<const uint32_t*>(x.ws.items);
  void* plan_args[] = {&x.desc, &x.num_series, &x.num_samples, &x.max_K, &x.chunk, &x.ws};
  void* grid_args[] = {&x.samples, &x.num_samples, &x.desc, &x.num_series, &x.prm, &x.max_K,
                       &x.out, &x.allU, &x.allU_len, &order};
  void* pers_args[] = {&x.samples, &x.num_samples, &x.desc, &x.num_series, &x.prm, &x.max_K,
                       &x.out, &x.allU, &x.allU_len, &x.chunk, &x.ws};
  void* fin_args[] = {&x.num_samples, &x.desc, &x.num_series, &x.prm, &x.max_K, &x.out,
                      &x.allU, &x.allU_len, &x.chunk, &x.ws};
  hipKernelNodeParams np[3] = {};
  int n = 0;
  np[n].blockDim = dim3(ks::kPlanNT);
  np[n].gridDim = dim3(1);
  np[n].func = reinterpret_cast<void*>(&ks::plan_kernel);
  np[n++].kernelParams = plan_args;
  uint32_t grid = x.num_series;
  if (mode == KS_LAUNCH_PERSISTENT) {
    if (int rc = persistent_grid(c, kc, v, grid)) return rc;
    np[n].blockDim = dim3(nt);
    np[n].gridDim = dim3(grid);
    np[n].func = const_cast<void*>(K.persistent);
    np[n++].kernelParams = pers_args;
    np[n].blockDim = dim3(nt);
    np[n].gridDim = dim3(x.num_series);
    np[n].func = const_cast<void*>(K.finish);
    np[n++].kernelParams = fin_args;
  } else {
    np[n].blockDim = dim3(nt);
    np[n].gridDim = dim3(x.num_series);
    np[n].func = const_cast<void*>(K.grid);
    np[n++].kernelParams = grid_args;
  }
  hipError_t e;
  if (!use_graph) {
    for (int i = 0; i < n; ++i) {
      e = hipLaunchKernel(np[i].func, np[i].gridDim, np[i].blockDim, np[i].kernelParams, 0, st);
      if (e != hipSuccess) return hip_fail(e, "plan launch");
    }
    return KS_OK;
  }
  // the graph topology depends on the grid sizes only through the nodes'
  // parameters, so one graph per (mode, K class, variant, persistent grid) is reused
  auto key = std::make_tuple(mode, kc, v, mode == KS_LAUNCH_PERSISTENT ? grid : 0u);
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    GraphEntry g;
    if ((e = hipGraphCreate(&g.graph, 0)) != hipSuccess) return hip_fail(e, "hipGraphCreate");
    for (int i = 0; i < n && e == hipSuccess; ++i)
      e = hipGraphAddKernelNode(&g.node[i], g.graph, i ? &g.node[i - 1] : nullptr, i ? 1 : 0, &np[i]);
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g.graph);
      return hip_fail(e, "graph build");
    }
    g.nodes = n;
    it = c->graphs.emplace(key, g).first;
  } else {
    for (int i = 0; i < n; ++i)
      if ((e = hipGraphExecKernelNodeSetParams(it->second.exec, it->second.node[i], &np[i])) != hipSuccess)
        return hip_fail(e, "graph update");
  }
  if ((e = hipGraphLaunch(it->second.exec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return KS_OK;
}

LaunchCfg config_for(const ks_ctx* c, int kc, uint32_t num_series, uint32_t opts) {
  LaunchCfg cfg;
  auto it = c->tuned.find(std::make_tuple(kc, num_series));
  if (it != c->tuned.end()) cfg = it->second;
  if (opts & KS_OPT_GRID) cfg.mode = KS_LAUNCH_GRID;
  if (opts & KS_OPT_PERSISTENT) cfg.mode = KS_LAUNCH_PERSISTENT;
  if (opts & KS_OPT_NO_GRAPH) cfg.graph = 0;
  return cfg;
}

int scan_with(ks_ctx* ctx, const ScanArgs& a, int kc, const LaunchCfg& cfg, hipStream_t st) {
  if (cfg.mode == KS_LAUNCH_GRID) {
    hipError_t e = launch_grid(kc, cfg.variant, a, st);
    return e == hipSuccess ? KS_OK : hip_fail(e, "scan launch");
  }
  const bool split = cfg.mode == KS_LAUNCH_PERSISTENT;
  if (int rc = ensure_workspace(ctx, a.num_series, split ? (uint64_t)a.num_series * a.max_K : 0)) return rc;
  ScanArgs b = a;
  b.chunk = split ? cfg.chunk_bytes : ks::kNoSplit;  // the ordered grid never splits
  b.ws = workspace_of(ctx);
  return launch_plan(ctx, kc, cfg.variant, cfg.mode, b, cfg.graph != 0, st);
}

bool valid_launch(const ks_launch* c) {
  return c && c->mode <= KS_LAUNCH_ORDERED && c->graph <= 1 && c->chunk_bytes >= 4096u &&
         c->chunk_bytes <= (1u << 30) && c->variant < (uint32_t)kNumVariants;
}

LaunchCfg from_launch(const ks_launch* c) {
  LaunchCfg l;
  l.mode = (int)c->mode;
  l.chunk_bytes = c->chunk_bytes;
  l.graph = (int)c->graph;
  l.variant = (int)c->variant;
  return l;
}

ks_launch to_launch(const LaunchCfg& l) {
  return ks_launch{(uint32_t)l.mode, l.chunk_bytes, (uint32_t)l.graph, (uint32_t)l.variant};
}

// Tune-cache lines: "<arch> <cus> <kclass> <num_series> <mode> <chunk_bytes> <graph> <variant>".
void load_tune_cache(ks_ctx* c) {
  const char* path = std::getenv("KS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[128];
  int cus, kc, pers, graph, var;
  unsigned ns, chunk;
  while (std::fscanf(f, "%127s %d %d %u %d %u %d %d", arch, &cus, &kc, &ns, &pers, &chunk, &graph, &var) == 8) {
    ks_launch l{(uint32_t)pers, chunk, (uint32_t)graph, (uint32_t)var};
    if (c->arch == arch && cus == c->num_cus && kc >= 0 && kc < kNumKClasses && var >= 0 && valid_launch(&l))
      c->tuned[std::make_tuple(kc, (uint32_t)ns)] = from_launch(&l);
  }
  std::fclose(f);
}

void append_tune_cache(const ks_ctx* c, int kc, uint32_t ns, const LaunchCfg& l) {
  const char* path = std::getenv("KS_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %u %d %u %d %d\n", c->arch.c_str(), c->num_cus, kc, ns, l.mode, l.chunk_bytes, l.graph,
               l.variant);
  std::fclose(f);
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
  {
    DeviceGuard g(device);
    if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
    if (int rc = resolve_scratch(device)) return rc;
  }
  ks_ctx* c = new (std::nothrow) ks_ctx();
  if (!c) return KS_E_NOMEM;
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  const size_t colon = c->arch.find(':');
  if (colon != std::string::npos) c->arch.resize(colon);
  load_tune_cache(c);
  *out = c;
  return KS_OK;
}

int ks_ctx_destroy(ks_ctx* ctx) {
  if (!ctx) return KS_E_INVALID;
  {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : ctx->graphs) {
      (void)hipGraphExecDestroy(kv.second.exec);
      (void)hipGraphDestroy(kv.second.graph);
    }
    free_workspace(ctx);
    free_learn(ctx->learn);
    free_seg(ctx->seg);
  }
  delete ctx;
  return KS_OK;
}

int ks_reserve(ks_ctx* ctx, uint32_t max_series, uint64_t max_total_steps) {
  if (!ctx) return KS_E_INVALID;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  return ensure_workspace(ctx, max_series, max_total_steps);
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
  const int kc = k_class(max_K);
  ScanArgs a{samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, 0, {}};
  return scan_with(ctx, a, kc, config_for(ctx, kc, num_series, params->opts), (hipStream_t)stream);
}

int ks_launch_set(ks_ctx* ctx, uint32_t max_K, uint32_t num_series, const ks_launch* cfg) {
  if (!ctx || !cfg) return KS_E_INVALID;
  if (!valid_launch(cfg)) return KS_E_RANGE;
  ctx->tuned[std::make_tuple(k_class(max_K ? max_K : KS_MAX_K), num_series)] = from_launch(cfg);
  return KS_OK;
}

int ks_launch_get(ks_ctx* ctx, uint32_t max_K, uint32_t num_series, ks_launch* cfg) {
  if (!ctx || !cfg) return KS_E_INVALID;
  *cfg = to_launch(config_for(ctx, k_class(max_K ? max_K : KS_MAX_K), num_series, 0));
  return KS_OK;
}

int ks_autotune(ks_ctx* ctx, const uint32_t* samples, uint64_t num_samples, const ks_desc* desc,
                uint32_t num_series, const ks_params* params, ks_result* out, void* stream, ks_launch* best,
                float* best_ms) {
  if (!ctx || !params || !out) return KS_E_INVALID;
  if (int rc = check_params(params)) return rc;
  if (num_series == 0) return KS_OK;
  if (!samples || !desc) return KS_E_INVALID;
  if (num_series > (1u << 30)) return KS_E_RANGE;
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const uint32_t max_K = params->max_K ? params->max_K : KS_MAX_K;
  const int kc = k_class(max_K);
  hipStream_t st = (hipStream_t)stream;
  ScanArgs a{samples, num_samples, desc, num_series, *params, max_K, out, nullptr, 0, 0, {}};
  hipEvent_t e0, e1;
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(e, "hipEventCreate");
  }
  // one warm-up (builds graphs, grows the workspace), then the best of three
  auto time_cfg = [&](const LaunchCfg& cfg, float& tmin) -> int {
    int rc = scan_with(ctx, a, kc, cfg, st);
    for (int r = 0; r < 3 && rc == KS_OK; ++r) {
      if ((e = hipEventRecord(e0, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
      if ((rc = scan_with(ctx, a, kc, cfg, st)) != KS_OK) return rc;
      if ((e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
        return hip_fail(e, "hipEventSynchronize");
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r == 0 || ms < tmin) tmin = ms;
    }
    return rc;
  };
  // every scan-kernel variant (tile, sort radix, walk window) under every
  // launch plan: the plain grid, the ordered grid from a hipGraph and direct,
  // the persistent queue with 1 / 4 / 16 MiB splits from a hipGraph and direct
  // (the variants rank differently under different plans)
  int rc = KS_OK;
  LaunchCfg bcfg;
  float bms = 0.f;
  bool have = false;
  for (int v = 0; v < kNumVariants && rc == KS_OK; ++v) {
    LaunchCfg plans[9];
    int np = 0;
    plans[np++] = LaunchCfg{KS_LAUNCH_GRID, 1u << 20, 0, v};
    plans[np++] = LaunchCfg{KS_LAUNCH_ORDERED, 1u << 20, 1, v};
    plans[np++] = LaunchCfg{KS_LAUNCH_ORDERED, 1u << 20, 0, v};
    for (uint32_t chunk : {1u << 20, 4u << 20, 16u << 20}) {
      plans[np++] = LaunchCfg{KS_LAUNCH_PERSISTENT, chunk, 1, v};
      plans[np++] = LaunchCfg{KS_LAUNCH_PERSISTENT, chunk, 0, v};
    }
    for (int i = 0; i < np && rc == KS_OK; ++i) {
      float t = 0.f;
      rc = time_cfg(plans[i], t);
      if (rc == KS_OK && (!have || t < bms)) {
        bcfg = plans[i];
        bms = t;
        have = true;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  ctx->tuned[std::make_tuple(kc, num_series)] = bcfg;
  append_tune_cache(ctx, kc, num_series, bcfg);
  if (best) *best = to_launch(bcfg);
  if (best_ms) *best_ms = bms;
  return KS_OK;
}

int ks_scan_batch_noalloc(ks_ctx* ctx, const uint32_t* samples, uint64_t num_samples, const ks_desc* desc,
                          uint32_t num_series, const ks_params* params, ks_result* out, uint32_t* all_U,
                          uint64_t all_U_len, void* stream) {
  if (!ctx || !params || !out) return KS_E_INVALID;
  if (int rc = check_params(params)) return rc;
  if (num_series == 0) return KS_OK;
  if (!samples || !desc) return KS_E_INVALID;
  if (num_series > KS_NOALLOC_MAX_SERIES) return KS_E_RANGE;
  unsigned char* base = scratch_of(ctx->device);
  if (!base) return KS_E_STATE;  // ks_ctx_create resolves it; not reached for a valid context
  DeviceGuard g(ctx->device);
  if (g.err != hipSuccess) return hip_fail(g.err, "hipSetDevice");
  const uint32_t max_K = params->max_K ? params->max_K : KS_MAX_K;
  const int kc = k_class(max_K);
  // the plan kernel rewrites the header, every item and every per-series word
  // it reads later, so nothing is cleared here
  ks::Workspace ws{reinterpret_cast<uint32_t*>(base), reinterpret_cast<ks::Item*>(base + kScratchItems),
                   reinterpret_cast<uint64_t*>(base + kScratchBase), reinterpret_cast<uint32_t*>(base + kScratchDone),
                   reinterpret_cast<uint32_t*>(base + kScratchMin), nullptr};
  ScanArgs a{samples, num_samples, desc, num_series, *params, max_K, out, all_U, all_U_len, ks::kNoSplit, ws};
  const int v = config_for(ctx, kc, num_series, 0).variant;  // the tuned kernel variant (a table lookup)
  return launch_plan(ctx, kc, v, KS_LAUNCH_ORDERED, a, false, (hipStream_t)stream);
}

}  // extern "C"

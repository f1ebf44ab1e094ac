// Host-side state shared by the library's translation units: the context,
// the model, error text and common validation.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <string>
#include <tuple>

#include "ks.h"

namespace ks {
struct Item;
struct RowMom;
}  // namespace ks

namespace ks_host {

constexpr int kNT = 256;
constexpr int kRB = 4;
constexpr int kNumKClasses = 6;
constexpr uint32_t kKClass[kNumKClasses] = {64, 128, 256, 512, 1024, 2048};

// Scan-kernel variants the autotuner chooses among (ks_launch.variant):
//   nt  workgroup size, i.e. the tile: waves streaming one series' rows and
//       sorting its keys (and, through the LDS each needs, how many series
//       stay resident per CU);
//   rb  bits of the key sort's radix digit (passes = key bits / rb);
//   gm  the walk window: 64-lane candidate slots a wave walks at once over the
//       sorted positions (0: its whole share, at most four).
// Variant 0 is the default. Each is instantiated for every K class and every
// launch mode (ks_scan_variants.hip, compiled once per variant).
struct Variant {
  int nt, rb, gm;
};
constexpr int kNumVariants = 6;
constexpr Variant kVariants[kNumVariants] = {{256, 4, 0}, {128, 4, 0}, {512, 4, 0},
                                             {256, 8, 0}, {256, 4, 1}, {256, 4, 2}};

// Kernels of one variant and K class: grid / ordered scan, persistent scan, finish.
struct ScanKernels {
  const void* grid;
  const void* persistent;
  const void* finish;
};
const ScanKernels& scan_kernels(int kclass, int variant);

inline int k_class(uint32_t max_K) {
  for (int i = 0; i < kNumKClasses; ++i)
    if (max_K <= kKClass[i]) return i;
  return kNumKClasses - 1;
}

// Launch configuration chosen per (K class) and batch size by the tuner.
struct LaunchCfg {
  int mode = KS_LAUNCH_ORDERED;  // KS_LAUNCH_GRID / _PERSISTENT / _ORDERED
  uint32_t chunk_bytes = 1u << 20;
  int graph = 1;                 // planned launches replayed from a hipGraph
  int variant = 0;               // kVariants index
};

struct GraphEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node[3] = {nullptr, nullptr, nullptr};
  int nodes = 0;
};

// Device buffers of the learned path, grown on demand.
struct LearnBuffers {
  // proposal pass (rows = num_series * SR)
  uint64_t* s1 = nullptr;
  uint64_t* s2lo = nullptr;
  uint32_t* s2hi = nullptr;
  uint32_t* smin = nullptr;
  uint32_t* K = nullptr;
  float* feat = nullptr;      // [rows][9]
  uint16_t* x0 = nullptr;     // [rows][16] bf16
  uint16_t* act[3] = {nullptr, nullptr, nullptr};  // [rows][64] bf16 (a1, a2, a3)
  float* logits = nullptr;    // [rows]
  // training
  uint16_t* dy16 = nullptr;   // [rows][16] bf16: logit gradient
  float* dy16f = nullptr;
  uint16_t* dy[3] = {nullptr, nullptr, nullptr};  // [rows][64] bf16: gradients at y2, y1, y0
  float* dyf[3] = {nullptr, nullptr, nullptr};     // the same in fp32 (before the bf16 rounding)
  float* part = nullptr;      // weight-gradient partials
  float* grad[4] = {nullptr, nullptr, nullptr, nullptr};  // reduced, per layer
  uint32_t* nsig = nullptr;
  uint64_t cap_rows = 0, cap_series = 0, cap_part = 0;
  // the last proposal / feature pass (ks_refine checks it)
  const void* stamp_desc = nullptr;
  uint32_t stamp_series = 0, stamp_SR = 0, stamp_maxK = 0;
  bool stamp_valid = false;
};

// Window workspace of the binary segmentation (ks_segment_batch), grown on demand.
struct SegBuffers {
  ks_desc* win[2] = {nullptr, nullptr};    // open windows of this / the next depth
  uint32_t* wser[2] = {nullptr, nullptr};  // their series
  uint32_t* wstart[2] = {nullptr, nullptr};  // their first row within the series
  ks_result* res = nullptr;                // scan results of the open windows
  uint32_t* ctr = nullptr;                 // device: per depth d, [2 d] its window count, [2 d + 1] their largest K
  uint32_t* host_ctr = nullptr;            // pinned host copy of ctr
  ks::RowMom* rows = nullptr;              // per-row moments and minimum of depth 0 (s * max_K + i)
  uint64_t cap = 0;                        // windows per buffer
  uint64_t cap_rows = 0;
};

int hip_fail(hipError_t e, const char* what);

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

inline int check_params(const ks_params* p) {
  if (!p) return KS_E_INVALID;
  if (!(p->alpha > 0.0 && p->alpha < 1.0)) return KS_E_INVALID;
  if (!(p->c_alpha > 0.0) || !std::isfinite(p->c_alpha)) return KS_E_INVALID;
  if (p->w < 1 || p->w > 64) return KS_E_INVALID;
  if (!(p->tau >= 0.0f && p->tau <= 1.0f)) return KS_E_INVALID;
  if (p->opts & ~(uint32_t)KS_OPT_MASK) return KS_E_INVALID;
  if (p->max_K != 0 && (p->max_K < 2 || p->max_K > KS_MAX_K)) return KS_E_RANGE;
  return KS_OK;
}

void free_learn(LearnBuffers& b);
void free_seg(SegBuffers& b);

}  // namespace ks_host

struct ks_ctx {
  int device = 0;
  int num_cus = 0;
  std::string arch;
  int occupancy[ks_host::kNumKClasses][ks_host::kNumVariants] = {};  // resident workgroups per CU of scan_persistent
  // scan workspace
  uint32_t* hdr = nullptr;
  ks::Item* items = nullptr;
  uint64_t* mom_base = nullptr;
  uint32_t* done = nullptr;
  uint32_t* smin = nullptr;
  ks::RowMom* mom = nullptr;
  uint64_t cap_series = 0, cap_rows = 0;
  std::map<std::tuple<int, int, int, uint32_t>, ks_host::GraphEntry> graphs;  // (mode, K class, variant, grid)
  std::map<std::tuple<int, uint32_t>, ks_host::LaunchCfg> tuned;         // (K class, num_series)
  ks_host::LearnBuffers learn;
  ks_host::SegBuffers seg;
};

struct ks_model {
  int device = 0;
  float* theta = nullptr;  // master weights, fp32
  float* m1 = nullptr;     // Adam moments
  float* m2 = nullptr;
  float* grad = nullptr;   // gradient of the last training step
  uint16_t* wf[4] = {nullptr, nullptr, nullptr, nullptr};
  uint16_t* wb[4] = {nullptr, nullptr, nullptr, nullptr};
  float* b[4] = {nullptr, nullptr, nullptr, nullptr};
  uint64_t step = 0;
};

/*
 * ks.h - C ABI of the MI355X (gfx950) Kolmogorov-Smirnov change-point library.
 *
 * The library detects the change point of latency-versus-footprint sweeps the
 * way MT4G does (arXiv 2511.05958, Section "Benchmarks and Autoevaluation",
 * size benchmarks, workflow step 4 "The K-S test"):
 *
 *   one series   = the 2-D timing array of one size sweep: K array sizes
 *                  (rows) x the first N load latencies of each size
 *                  (columns), uint32 cycles, row-major;
 *   reduction    = eq. 2, S_i = sqrt(sum_j (r_ij - min r)^2), min r over the
 *                  whole array; kept exactly as Q_i = S_i^2 (K-S needs ranks
 *                  only, and sqrt is strictly increasing);
 *   candidates   = every row index c in [1, K-1]; lower side rows [0, c)
 *                  (n = c values), higher side rows [c, K) (m = K - c values);
 *   statistic    = two-sample K-S, D_c = max_x |F(x) - G(x)| (Section
 *                  "Background", K-S test), kept as the integer
 *                  U_c = n m D_c = max |i m - j n| over complete tie groups;
 *   choice       = the most significant candidate: largest
 *                  lambda_c = D_c sqrt(n m / (n + m)), ties to the smaller c;
 *   significance = eq. 1 with the sign fixed, d_alpha^2 = c_alpha (n+m)/(n m),
 *                  c_alpha = -1/2 ln(alpha/2); H0 denied iff D > d_alpha,
 *                  evaluated as U^2 > c_alpha n m K in IEEE double;
 *   confidence   = asymptotic Kolmogorov p-value Q_KS(lambda) of the winner.
 *
 * Conventions for every entry point:
 *   - Status: KS_OK (0) or a negative KS_E_* code; ks_status_string() names it.
 *     A KS_E_HIP return keeps the HIP error text of the calling thread for
 *     ks_status_string(KS_E_HIP).
 *   - Memory: arguments documented as "device" are device pointers owned by
 *     the caller; the library never frees or retains them past the call's
 *     stream work. "host" arguments are read during the call only.
 *   - Streams: `stream` is a hipStream_t of the context's device (NULL = the
 *     null stream). Calls are asynchronous and stream-ordered; results are
 *     valid once the stream's work up to the call has completed.
 *   - Contexts are not thread-safe: use one ks_ctx per host thread. The calls
 *     of one context share its device workspace, so they must be ordered on
 *     one stream (or the caller waits between streams).
 */
#ifndef KS_H
#define KS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KS_VERSION 10000 /* 1.0.0 */

#define KS_MAX_K 2048u          /* rows per series */
#define KS_MAX_N (1u << 24)     /* samples per row */

/* status codes */
#define KS_OK 0
#define KS_E_INVALID (-1) /* null pointer, bad parameter */
#define KS_E_RANGE (-2)   /* a size outside the documented limits */
#define KS_E_STATE (-3)   /* call order / workspace stamp mismatch */
#define KS_E_HIP (-4)     /* a HIP runtime call failed */
#define KS_E_MODEL (-5)   /* bad model handle, file or weights */
#define KS_E_NOMEM (-6)   /* device allocation failed */

/* ks_result.flags */
#define KS_SIGNIFICANT 1u    /* H0 denied at alpha (eq. 1) */
#define KS_REFINED 2u        /* ks_refine: exact scan inside the +-w window */
#define KS_FALLBACK 4u       /* ks_refine: low confidence, full exact scan */
#define KS_BAD_SHAPE 8u      /* K < 2, K > max_K, N < 1 or N > KS_MAX_N; cp = 0 */
#define KS_OUT_OF_RANGE 16u  /* offset + K*N exceeds num_samples; cp = 0 */

/* One series of the batch. 24 bytes; an array of these lives in device memory.
 *   offset      first sample of the series, in uint32 elements from `samples`
 *   K, N        rows and samples per row; the series is samples[offset + i*N + j]
 *   aux_offset  first slot of this series in the optional per-row outputs
 *               (all_U), normally the sum of K over the preceding series */
typedef struct ks_desc {
  uint64_t offset;
  uint32_t K;
  uint32_t N;
  uint64_t aux_offset;
} ks_desc;

/* Result of one series. 48 bytes.
 *   cp      c*, the first row of the higher side (the change point); the
 *           cache size lies between footprint[cp-1] and footprint[cp]
 *   n, m    side sizes c* and K - c*
 *   U       D numerator n m D (exact integer)
 *   D       U / (n m)
 *   lambda  sqrt(U^2 / (n m K))
 *   p       asymptotic Kolmogorov p-value of lambda (FP64); 1 when U = 0,
 *           0 when 2 lambda^2 > 700
 *   flags   KS_* flags above */
typedef struct ks_result {
  uint32_t cp, n, m, U;
  double D, lambda, p;
  uint32_t flags, pad;
} ks_result;

/* Method and launch parameters. 32 bytes.
 *   alpha    significance level in (0, 1)
 *   c_alpha  -1/2 ln(alpha/2), filled by ks_params_init on the host so every
 *            decision uses the same bits
 *   max_K    upper bound on K over the batch (2..KS_MAX_K, 0 = KS_MAX_K);
 *            sizes the per-workgroup LDS; series with K > max_K get
 *            KS_BAD_SHAPE
 *   w        refine half-window (ks_refine), 1..64, default 8
 *   tau      confidence threshold of ks_refine in [0, 1]; below it the full
 *            scan runs (default 0.5)
 *   opts     KS_OPT_* launch overrides (0 = the tuned or default plan) */
typedef struct ks_params {
  double alpha;
  double c_alpha;
  uint32_t max_K;
  uint32_t w;
  float tau;
  uint32_t opts;
} ks_params;

/* ks_params.opts: launch overrides, for measurement and tuning. */
#define KS_OPT_GRID 1u        /* force KS_LAUNCH_GRID */
#define KS_OPT_PERSISTENT 2u  /* force KS_LAUNCH_PERSISTENT */
#define KS_OPT_NO_GRAPH 4u    /* launch the plan's kernels directly instead of a hipGraph */
#define KS_OPT_MASK 7u

typedef struct ks_ctx ks_ctx;

/* KS_VERSION of the built library. */
int ks_version(void);

/* Static text for a status code (for KS_E_HIP, the calling thread's last HIP
 * error text). Never NULL. */
const char *ks_status_string(int status);

/* Fill *p with alpha, c_alpha = -1/2 ln(alpha/2) (eq. 1 with the sign
 * fixed), max_K = 0, w = 8, tau = 0.5, opts = 0. KS_E_INVALID if p is NULL
 * or alpha is not in (0, 1). */
int ks_params_init(ks_params *p, double alpha);

/* Create a context on HIP device `device`: device properties, workspace,
 * graph cache and tuning table. *out owns them until ks_ctx_destroy. */
int ks_ctx_create(int device, ks_ctx **out);
int ks_ctx_destroy(ks_ctx *ctx);

/* Pre-allocate workspace for batches of up to max_series series and
 * max_total_steps total rows, so that later calls of that size allocate
 * nothing. Optional; calls grow the workspace on demand otherwise. */
int ks_reserve(ks_ctx *ctx, uint32_t max_series, uint64_t max_total_steps);

/* Exact scan of a batch (eq. 2 reduction, K-S at every candidate, choice,
 * significance, p-value) for every series.
 *   samples      device, uint32[num_samples]
 *   desc         device, ks_desc[num_series]
 *   params       host, read during the call
 *   out          device, ks_result[num_series]
 *   all_U        device, nullable: uint32[all_U_len]; series s writes
 *                all_U[aux_offset + c] = U_c for c in [0, K) (U_0 = 0) when
 *                aux_offset + K <= all_U_len, and nothing otherwise
 * num_series == 0 is a no-op. Per-series shape or range errors are reported
 * in out[s].flags (cp = 0), not as a status. KS_E_INVALID on a NULL pointer
 * or a bad alpha / c_alpha / w / tau / opts, KS_E_RANGE on max_K outside
 * [2, KS_MAX_K] (0 allowed), KS_E_NOMEM if the workspace cannot grow.
 *
 * Launch plan (ks_launch_set / ks_autotune; default KS_LAUNCH_ORDERED): an
 * on-device planning kernel orders the series largest first, then either one
 * workgroup per series in that order, or a persistent kernel drains the
 * ordered items (large series split into row ranges whose moments meet in
 * the workspace) followed by a finish kernel. Planned launches are replayed
 * from a hipGraph cached per (mode, max_K class, grid) with updated
 * arguments. The workspace grows on demand (that growth synchronizes the
 * device); ks_reserve avoids it. */
int ks_scan_batch(ks_ctx *ctx, const uint32_t *samples, uint64_t num_samples, const ks_desc *desc,
                  uint32_t num_series, const ks_params *params, ks_result *out, uint32_t *all_U,
                  uint64_t all_U_len, void *stream);

/* ks_launch.mode */
#define KS_LAUNCH_GRID 0u        /* one workgroup per series, descriptor order, no plan */
#define KS_LAUNCH_PERSISTENT 1u  /* plan + persistent queue over (split) items + finish kernel */
#define KS_LAUNCH_ORDERED 2u     /* plan + one workgroup per series, largest series first */

/* Launch plan for one batch shape (max_K class, num_series).
 *   mode         KS_LAUNCH_*
 *   chunk_bytes  split size of KS_LAUNCH_PERSISTENT, 4 KiB .. 1 GiB: series
 *                with more sample bytes are cut into row ranges of about
 *                this size (at most 64 per series)
 *   graph        1: replay a planned launch from a cached hipGraph;
 *                0: launch its kernels directly
 *   variant      scan-kernel variant, 0 .. KS_SCAN_VARIANTS - 1 (tile = the
 *                workgroup size, radix digit bits of the key sort, walk
 *                window = candidate slots of 64 a wave walks at once):
 *                0 {256 threads, 4 bits, whole share}, 1 {128, 4, share},
 *                2 {512, 4, share}, 3 {256, 8, share}, 4 {256, 4, one slot},
 *                5 {256, 4, two slots}. Every variant gives the same results. */
#define KS_SCAN_VARIANTS 6u
typedef struct ks_launch {
  uint32_t mode;
  uint32_t chunk_bytes;
  uint32_t graph;
  uint32_t variant;
} ks_launch;

/* Record (ks_launch_set) or read (ks_launch_get) the plan ks_scan_batch uses
 * for batches with this max_K class and num_series; without a record the
 * default is {KS_LAUNCH_ORDERED, 1 MiB, 1, 0}. KS_E_INVALID / KS_E_RANGE on
 * bad values. */
int ks_launch_set(ks_ctx *ctx, uint32_t max_K, uint32_t num_series, const ks_launch *cfg);
int ks_launch_get(ks_ctx *ctx, uint32_t max_K, uint32_t num_series, ks_launch *cfg);

/* Autotuner, on this very batch with HIP events on `stream` (one warm-up,
 * best of three per candidate): every scan-kernel variant (tile, sort radix,
 * walk window) under every launch plan (grid; ordered grid from a hipGraph and
 * direct; persistent with chunk_bytes 1, 4, 16 MiB, from a hipGraph and
 * direct), 6 x 9 candidates. Records the fastest
 * with ks_launch_set and returns it in *best (nullable) and its time in
 * *best_ms (nullable). Blocks until done; writes `out`. When the environment
 * variable KS_TUNE_CACHE names a file, the choice is appended to it, and
 * ks_ctx_create loads the records written for the same device (architecture
 * and CU count). Arguments as ks_scan_batch. */
int ks_autotune(ks_ctx *ctx, const uint32_t *samples, uint64_t num_samples, const ks_desc *desc,
                uint32_t num_series, const ks_params *params, ks_result *out, void *stream, ks_launch *best,
                float *best_ms);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ks_scan_batch
 * with the ordered launch plan (largest series first, one workgroup per
 * series), run on a fixed scratch array in the library's device image
 * instead of the context's workspace. It allocates nothing and launches the
 * plan's two kernels directly (no hipGraph).
 *   Arguments, results and per-series flags as ks_scan_batch; params->opts
 *   is checked but the launch plan is always the ordered grid (with the
 *   scan-kernel variant recorded for this batch shape, else variant 0).
 *   num_series <= KS_NOALLOC_MAX_SERIES, else KS_E_RANGE (nothing launched).
 *   Scratch: 256 + 24 * KS_NOALLOC_MAX_SERIES bytes (12 MiB + 256 B) per
 *   device, held until the process ends; ks_ctx_create resolves its address
 *   on the context's device. Every call on one device shares it and each
 *   call's planning kernel rewrites what the call reads, so calls in
 *   sequence on any streams of one device are fine, but calls whose work
 *   overlaps in time on one device race on the scratch and give undefined
 *   results: order them on one stream, or wait between streams. */
#define KS_NOALLOC_MAX_SERIES (1u << 19)
int ks_scan_batch_noalloc(ks_ctx *ctx, const uint32_t *samples, uint64_t num_samples, const ks_desc *desc,
                          uint32_t num_series, const ks_params *params, ks_result *out, uint32_t *all_U,
                          uint64_t all_U_len, void *stream);

/* ------------------------------------------------------------------------
 * Learned proposal (not in the paper: the paper notes that candidate change
 * points could be shortlisted to save work and skips it because its data are
 * small; workflow step 4, last paragraph). A small network proposes the
 * change point of each series from per-row decile features; the exact K-S
 * choice then runs only within +-w rows of the proposal (ks_refine), or over
 * all candidates when the proposal's confidence is below tau.
 *
 * Network: conv(11->64) ReLU, conv(64->64) ReLU, conv(64->64) ReLU,
 * conv(64->1), kernel 5, zero padding 2, bias; one logit per row; bf16
 * operands on the matrix cores with fp32 accumulation. Input channels of row
 * t: the nine features, t / (K-1) and 4 t (K - t) / K^2 (double, rounded to
 * float; the K-S choice favours central splits). Parameters (KS_CNN_PARAMS
 * fp32 values, in this order): W0[64][11][5] b0[64] W1[64][64][5] b1[64]
 * W2[64][64][5] b2[64] W3[1][64][5] b3[1].
 * Features: for row i the nine deciles x_(floor(k (N-1)/10)), k = 1..9, of
 * the row's samples, f = (double)(x - m) / max(m, 1) rounded to float, m the
 * series minimum; layout float[row][9] with series s at rows aux_offset.. .
 * ------------------------------------------------------------------------ */

#define KS_CNN_PARAMS 44993u
/* Largest N the feature and statistics passes accept: every row length the
 * scan accepts. Rows of up to 4096 + 3 samples are held in registers; longer
 * rows are streamed through the same order-statistics select. */
#define KS_FEATURE_MAX_N KS_MAX_N

typedef struct ks_model ks_model;

/* Create a model on ctx's device: He-uniform weights drawn from `seed`
 * (splitmix64), zero biases, zero Adam state. */
int ks_model_create(ks_ctx *ctx, uint64_t seed, ks_model **out);
int ks_model_destroy(ks_model *model);

/* Copy the master parameters in (host float[KS_CNN_PARAMS]; resets the Adam
 * state and step; KS_E_MODEL on a non-finite value) or out. */
int ks_model_set_params(ks_model *model, const float *params);
int ks_model_get_params(ks_model *model, float *params);

/* Host copy of the gradient computed by the last ks_train_step (same layout). */
int ks_model_grads(ks_model *model, float *grads);

/* Checkpoint file: "KSCNN001", parameter count, step, parameters, both Adam
 * moments, FNV-1a 64 checksum. ks_model_load returns KS_E_MODEL on a bad
 * magic, size or checksum. Synchronous. */
int ks_model_save(ks_model *model, const char *path);
int ks_model_load(ks_model *model, const char *path);

/* Pre-allocate the learned-path workspace (per-row moments, features,
 * activations, logits; the training buffers too when `train` is nonzero) for
 * batches of up to max_series series with K <= max_K (0 = KS_MAX_K), so that
 * ks_features, ks_propose, ks_refine and the network calls of that size
 * allocate nothing. Optional: those calls grow the workspace on demand, but a
 * caller that reserves before loading its samples also keeps the per-row
 * buffers apart from the sample allocation. KS_E_RANGE for max_K outside
 * [2, KS_MAX_K] or max_series above 2^26, KS_E_NOMEM when the device is full
 * (the workspace is then empty). Synchronises the device when it grows. */
int ks_learn_reserve(ks_ctx *ctx, uint32_t max_series, uint32_t max_K, int train);

/* Feature pass: per-row moments kept in the context (for ks_refine) and
 * decile features, written to `features` (device, nullable, float[rows][9],
 * series s at rows aux_offset .. aux_offset + K - 1 when they fit in
 * feature_rows). Series with K > max_K (0 = KS_MAX_K), N > KS_FEATURE_MAX_N
 * or a bad shape / range are skipped. */
int ks_features(ks_ctx *ctx, const uint32_t *samples, uint64_t num_samples, const ks_desc *desc,
                uint32_t num_series, uint32_t max_K, float *features, uint64_t feature_rows, void *stream);

/* Network forward on caller features (device float[feature_rows][9] at
 * aux_offset): logits (device float[logit_rows], row aux_offset + t). */
int ks_cnn_forward(ks_ctx *ctx, const ks_model *model, const float *features, uint64_t feature_rows,
                   const ks_desc *desc, uint32_t num_series, uint32_t max_K, float *logits, uint64_t logit_rows,
                   void *stream);

/* Proposal: the feature pass, the network, then per series
 * proposal[s] = argmax of the logits over rows 1..K-1 (smallest on ties) and
 * confidence[s] = softmax mass of the rows within +-params->w of it (device
 * int32 / float arrays of num_series). Skipped series get proposal 0,
 * confidence 0. features: as ks_features (nullable).
 * model == NULL proposes without a network (the baseline a trained network is
 * measured against): the row t in 1..K-1 with the largest |f_t - f_(t-1)| of
 * the per-row median (feature 5), ties to the smaller t, confidence 1. */
int ks_propose(ks_ctx *ctx, const ks_model *model, const uint32_t *samples, uint64_t num_samples,
               const ks_desc *desc, uint32_t num_series, const ks_params *params, int32_t *proposal,
               float *confidence, float *features, uint64_t feature_rows, void *stream);

/* Exact refine after ks_propose (or ks_features) on the same stream with the
 * same desc pointer, num_series and max_K (else KS_E_STATE): for each series
 * the full scan's choice restricted to candidates max(1, p-w) .. min(K-1, p+w)
 * when confidence >= tau (flag KS_REFINED), or over all candidates otherwise
 * (KS_FALLBACK; also for a NaN confidence or an empty window). Reads only the
 * moments kept by the feature pass, not the samples. num_samples as given to
 * that pass (for the same shape / range checks). */
int ks_refine(ks_ctx *ctx, const ks_desc *desc, uint32_t num_series, uint64_t num_samples, const int32_t *proposal,
              const float *confidence, const ks_params *params, ks_result *out, void *stream);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected, fp32 master
 * weights, bf16 copies rebuilt) on the mean softmax cross-entropy over rows
 * 1..K-1 of the series whose label (device int32[num_series]) is >= 1; label
 * -1 skips a series. features as ks_cnn_forward. loss: device float, nullable
 * (the batch's mean loss before the update). */
int ks_train_step(ks_ctx *ctx, ks_model *model, const float *features, uint64_t feature_rows, const ks_desc *desc,
                  const int32_t *labels, uint32_t num_series, uint32_t max_K, float lr, float *loss, void *stream);

/* Gradient, at the model's current weights, of L = sum over series s and rows
 * t < K_s of dlogits[aux_offset + t] * logit[aux_offset + t]: the training
 * step's forward and backward passes (same kernels, same bf16 rounding of the
 * layer inputs, weights and output gradients, fp32 accumulation), with the
 * logit gradient given by the caller instead of the softmax cross-entropy's.
 * For other losses of the logits (pass dL/dlogit), and for checking the
 * backward pass on its own.
 *   features  device float[feature_rows][9], as ks_cnn_forward
 *   dlogits   device float[dlogit_rows], row aux_offset + t of series s;
 *             a series whose rows do not fit in dlogit_rows contributes 0
 *   grads     device float[KS_CNN_PARAMS], written in the parameter layout
 * The weights, the Adam state and the gradient kept for ks_model_grads are not
 * changed. Skipped series (K > max_K or a bad shape) contribute nothing;
 * num_series == 0 writes a zero gradient. KS_E_INVALID on a NULL pointer,
 * KS_E_RANGE on max_K outside [2, KS_MAX_K], KS_E_NOMEM if the training
 * buffers cannot grow. */
int ks_cnn_backward(ks_ctx *ctx, const ks_model *model, const float *features, uint64_t feature_rows,
                    const ks_desc *desc, uint32_t num_series, uint32_t max_K, const float *dlogits,
                    uint64_t dlogit_rows, float *grads, void *stream);

/* The network's intermediate values, for checking each layer on its own
 * inputs: the training step's forward pass (one kernel per layer) on caller
 * features and, when labels or dlogits is given, its backward pass.
 *   labels     device int32[num_series], nullable: when given, the logit
 *              gradient is the training step's (softmax cross-entropy, label
 *              -1 skips a series); otherwise
 *   dlogits    device float[dlogit_rows], nullable: the caller's logit
 *              gradient as for ks_cnn_backward
 *   acts       device, nullable, float[trace_rows][KS_CNN_TRACE_ACTS]: row
 *              aux_offset + t of series s holds the bf16 network input x0[11],
 *              the bf16 activations a1[64], a2[64], a3[64] (as floats) and the
 *              fp32 logit
 *   grads_in   device, nullable, float[trace_rows][KS_CNN_TRACE_GRADS]: the
 *              fp32 logit gradient, then the fp32 gradients at the
 *              pre-activations y2, y1, y0 [64 each] (masked by ReLU; the next
 *              layer down takes their bf16 roundings)
 *   grads      device, nullable, float[KS_CNN_PARAMS]: the parameter gradient
 * A series is written only when aux_offset + K <= trace_rows. The model is not
 * changed. KS_E_INVALID on a NULL pointer, or grads_in / grads without labels
 * or dlogits; KS_E_RANGE on max_K outside [2, KS_MAX_K]. */
#define KS_CNN_TRACE_ACTS 204u
#define KS_CNN_TRACE_GRADS 193u
int ks_cnn_trace(ks_ctx *ctx, const ks_model *model, const float *features, uint64_t feature_rows,
                 const ks_desc *desc, uint32_t num_series, uint32_t max_K, const int32_t *labels,
                 const float *dlogits, uint64_t dlogit_rows, float *acts, float *grads_in, uint64_t trace_rows,
                 float *grads, void *stream);

/* ------------------------------------------------------------ segmentation */

/* Every level boundary of each series, by binary segmentation. The paper's
 * test finds one change point per application, on a search interval narrowed
 * until one boundary is isolated (workflow steps 2-4); here the test is
 * applied to the whole series and then again to both sides [a, c) and [c, b)
 * of every window whose split c is significant. Each window is a series of
 * its own: eq. 2 with the window's own global minimum, every index a
 * candidate, eq. 1 significance. A window of fewer than 2 rows, or a
 * non-significant one, ends its branch; windows of depth d (0 = the whole
 * series) are scanned while max_levels == 0 or d < max_levels.
 *   desc        device, ks_desc[num_series] (aux_offset is ignored)
 *   params      host, as for ks_scan_batch (max_K bounds every K)
 *   max_levels  0 = until no window splits; 1 = the plain scan's split only
 *   max_cp      capacity per series of cps (>= 1; K - 1 always suffices)
 *   cps         device, ks_result[num_series * max_cp]: the boundaries of
 *               series s at cps[s * max_cp ...], sorted by cp, where cp
 *               counts rows from row 0 of the series; n = cp - a and m = b - cp
 *               for the boundary's window [a, b); U, D, lambda, p and flags
 *               are that window's; pad holds the window's depth
 *   counts      device, uint32[num_series]: boundaries found for series s.
 *               Above max_cp only max_cp of them are stored (which ones is
 *               unspecified). 0xffffffff for a series whose descriptor
 *               ks_scan_batch would flag KS_BAD_SHAPE or KS_OUT_OF_RANGE.
 * The depths run breadth-first: one ks_scan_batch over all open windows per
 * depth. Between depths the call reads back the next depth's window count
 * and largest K, which synchronizes `stream` once per depth. The window
 * workspace (num_series * max(1, max_K / 2) windows, 80 B each) grows on
 * demand. KS_E_INVALID on a NULL pointer, max_cp == 0 or a bad parameter,
 * KS_E_RANGE / KS_E_NOMEM as ks_scan_batch. */
int ks_segment_batch(ks_ctx *ctx, const uint32_t *samples, uint64_t num_samples, const ks_desc *desc,
                     uint32_t num_series, const ks_params *params, uint32_t max_levels, uint32_t max_cp,
                     ks_result *cps, uint32_t *counts, void *stream);

#define KS_SEGMENT_BAD 0xffffffffu /* ks_segment_batch counts[s] of a malformed series */

/* ---------------------------------------------------- per-row statistics */

/* Latency statistics of one row (one array size's N measurements): the
 * average as the main result, with p50, p95 and the standard deviation
 * beside it (Section "Load Latency benchmarks"), plus the minimum and
 * maximum. 32 bytes.
 *   mean     (sum r) / N: one FP64 division of the exact integer sum
 *   std      population standard deviation: num = N sum r^2 - (sum r)^2
 *            exact in 128 bits, rounded once to FP64, divided by N^2 in
 *            FP64, FP64 square root
 *   min, p50, p95, max   x_(floor(q (N - 1))) of the row sorted ascending,
 *            for q = 0, 0.5, 0.95, 1 */
typedef struct ks_row_stats {
  double mean;
  double std;
  uint32_t min, p50, p95, max;
} ks_row_stats;

/* Statistics of every row of every series, in one read of the samples.
 *   desc      device, ks_desc[num_series]; series s writes its rows to
 *             out[aux_offset + i], i < K, when aux_offset + K <= out_rows
 *   max_K     upper bound on K (0 = KS_MAX_K), as for ks_scan_batch
 *   out       device, ks_row_stats[out_rows]
 * A series that ks_scan_batch would flag (KS_BAD_SHAPE, KS_OUT_OF_RANGE), or
 * with N > KS_FEATURE_MAX_N, writes mean = std = NaN and zeros for its rows.
 * The series' order per row class (longest first) is kept in the context's
 * scan workspace, which grows to num_series series as with ks_reserve
 * (KS_E_NOMEM when the device is full).
 * KS_E_INVALID on a NULL pointer, KS_E_RANGE on max_K outside [2,
 * KS_MAX_K]. */
int ks_stats_batch(ks_ctx *ctx, const uint32_t *samples, uint64_t num_samples, const ks_desc *desc,
                   uint32_t num_series, uint32_t max_K, ks_row_stats *out, uint64_t out_rows, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KS_H */

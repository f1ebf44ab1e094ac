/* What the measurement workflow does around one detection (libks.so):
 * the outlier check and interval widening of workflow step 3 (Section "Size
 * benchmarks"), the L2 segment size aligned to an integer fraction of the
 * reported size (Section "L2 segment size") and the cache-line-size scoring
 * (Section "Cache Line Size benchmarks"). The paper states the goals but no
 * rule, weight or threshold; the readings are spelled out at each entry
 * point. Every entry point is asynchronous on `stream` (a hipStream_t, NULL
 * for the default stream) and returns KS_OK, KS_E_INVALID (-1) on a NULL
 * pointer or a bad parameter, KS_E_RANGE (-2) on a size outside the stated
 * limits, KS_E_HIP (-4) if a launch fails. */
#ifndef KS_SWEEP_H
#define KS_SWEEP_H

#include <stdint.h>

#include "ks.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------ workflow step 3 */

#define KS_CHECK_EDGE_LOW 1u     /* fewer than `edge` steps below the change point */
#define KS_CHECK_EDGE_HIGH 2u    /* fewer than `edge` steps from the change point up */
#define KS_CHECK_NO_CHANGE 4u    /* the test is not significant */
#define KS_CHECK_DISTURBED 8u    /* at least one disturbed step */
#define KS_CHECK_INVALID 0x80000000u /* malformed descriptor or flagged result; other fields 0 */

/* One sweep's check. 32 bytes.
 *   flags        KS_CHECK_*
 *   disturbed    number of disturbed steps
 *   lo, hi       the interval to measure next, in steps of the current one
 *                [0, K): [0, K) when nothing was found
 *   med_lo/hi    lower median of the steps' p50 latencies below / from the
 *                change point (both: the whole sweep when not significant)
 *   mad_lo/hi    lower median of their absolute deviations from it */
typedef struct ks_check {
  uint32_t flags, disturbed;
  int32_t lo, hi;
  uint32_t med_lo, med_hi, mad_lo, mad_hi;
} ks_check;

/* Outlier check and widening of every sweep (series) of a batch, from its
 * detection and its per-step statistics. The reading:
 *   - the sides are the steps [0, cp) and [cp, K) of a significant result,
 *     the whole sweep otherwise; a side's level is the lower median
 *     x_(floor((n - 1) / 2)) of its steps' p50, its spread the lower median
 *     of |p50 - level| (MAD);
 *   - a step is disturbed when |p50 - level| > k max(MAD, max(1, level / 64))
 *     (exact integers, level / 64 rounded down);
 *   - the change point is close to a boundary when a side has fewer than
 *     `edge` steps;
 *   - widening: no significant change -> [-K, 2K); close to the low (high)
 *     end -> lo = -K (hi = 2K); any disturbed step -> lo <= -(K / 2) and
 *     hi >= K + K / 2 (K / 2 rounded down).
 *   desc      device, ks_desc[num_series]: K and aux_offset are read
 *   res       device, ks_result[num_series] from ks_scan_batch (cp, flags)
 *   stats     device, ks_row_stats[stats_rows] from ks_stats_batch: step i
 *             of series s at stats[aux_offset + i]
 *   edge, k   >= 1 (defaults 4 and 5)
 *   out       device, ks_check[num_series]
 * A series with K < 2 or K > max_K (0 = KS_MAX_K), steps past stats_rows, or
 * a result flagged KS_BAD_SHAPE / KS_OUT_OF_RANGE gets KS_CHECK_INVALID. */
int ks_check_batch(ks_ctx *ctx, const ks_desc *desc, uint32_t num_series, uint32_t max_K, const ks_result *res,
                   const ks_row_stats *stats, uint64_t stats_rows, uint32_t edge, uint32_t k, ks_check *out,
                   void *stream);

/* ------------------------------------------------ L2 segment size */

/* Aligns benchmarked segment sizes to integer fractions of the reported
 * total: item i gets the k >= 1 minimising |S - T / k| (ties to the smaller
 * k), the aligned size T / k and the distance |S k - T| / T, which is
 * |S - T / k| relative to T / k and serves as the confidence (0 = exact).
 * The two ratios are one correctly rounded FP64 division of exact integers
 * each.
 *   measured, total   device, uint64_t[n], bytes, 1 <= S, T < 2^50 and
 *                     T / S < 2^32 - 16 (rounded down)
 *   segments          device, uint32_t[n] (k; 0 for an item out of range)
 *   aligned, distance device, double[n] (NaN for an item out of range) */
int ks_align_batch(const uint64_t *measured, const uint64_t *total, uint32_t n, uint32_t *segments,
                   double *aligned, double *distance, void *stream);

/* ------------------------------------------------ cache line size */

#define KS_LINE_INCONCLUSIVE 1u  /* fewer than two power-of-two strides */
#define KS_LINE_NO_INCREASE 2u   /* the score does not increase between them */
#define KS_LINE_NO_MAX_LIKE 4u   /* no stride more similar to MAX than to the pivot */
#define KS_LINE_INVALID 0x80000000u

/* One experiment's result. 24 bytes.
 *   line    the line size in bytes (0 when inconclusive or invalid)
 *   jstar   the first stride index scored more similar to MAX (J if none)
 *   jump    the largest score increase, as a fraction of the largest score */
typedef struct ks_line {
  uint32_t line, jstar, flags, pad;
  double jump;
} ks_line;

/* Cache-line-size scoring of every experiment of a batch. Experiment e is a
 * series of K = J A rows (rows j A .. j A + A - 1 hold stride j at the array
 * sizes a = 0 .. A - 1, ascending, around and above the cache size); its p50
 * latencies x[j][a] come from ks_stats_batch (stats[aux_offset + j A + a]).
 * Stride 0 is the pivot (surely below the line size), stride J - 1 the MAX
 * (surely above). The reading:
 *   - dp = |x - x[0][a]|, dm = |x - x[J-1][a]|, q = floor(2^32 dp / (dp + dm))
 *     (0 when both are 0): 0 is pivot-like, 2^32 MAX-like;
 *   - score_j = sum_a (a + 1) q_j(a), exact: larger arrays weigh more;
 *   - jstar = the first j >= 1 whose score exceeds half of W 2^32, W =
 *     sum_a (a + 1); from jstar on the score is its running maximum (an
 *     aliased stride looking like the pivot again does not count);
 *   - over the strides that are powers of two, in order, the largest increase
 *     of that score between consecutive ones, ties to the first; the line
 *     size is the stride before it.
 *   desc     device, ks_desc[num_exp]: K = J A and aux_offset are read
 *   stats    device, ks_row_stats[stats_rows]
 *   strides  device, uint32_t[J], bytes, ascending
 *   out      device, ks_line[num_exp]
 * J in [2, 64], A in [1, 256]; an experiment with K != J A, or rows past
 * stats_rows, gets KS_LINE_INVALID. */
int ks_line_batch(ks_ctx *ctx, const ks_desc *desc, uint32_t num_exp, const ks_row_stats *stats, uint64_t stats_rows,
                  uint32_t J, const uint32_t *strides, ks_line *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KS_SWEEP_H */

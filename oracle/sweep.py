"""CPU oracle, part 2: what the workflow does around one detection.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: plain Python integers over
one sweep at a time, written from the paper's description and the readings
below; the GPU path shares no code with it.

* ``check_sweep``  workflow step 3 (Section "Size benchmarks"): the results of
                   a sweep are checked for outliers, notably a cache size close
                   to a boundary of the search interval or a disturbed
                   measurement; if any is found the interval is widened and
                   the sweep repeated. The paper gives no rule; the reading:
      - the sides are the steps below and from the detected change point (the
        whole sweep when the test is not significant);
      - each side's level is the lower median of its steps' p50 latencies,
        its spread the lower median of the absolute deviations from it (MAD);
      - a step is disturbed when its deviation exceeds k max(MAD, floor),
        floor = max(1, level // 64), all in exact integers;
      - the change point is close to a boundary when a side has fewer than
        `edge` steps;
      - widening, in steps of the current interval [0, K): no significant
        change -> [-K, 2K); close to the low (high) end -> the low (high) end
        moves out by K; any disturbed step -> at least [-(K // 2), K + K // 2).
* ``align_fraction``  the L2 segment size (Section "L2 segment size"): a
                   benchmarked size S is aligned to the nearest integer
                   fraction T / k (k >= 1) of the reported size T; the distance
                   |S - T / k| / (T / k) = |S k - T| / T is the confidence.
* ``line_size``    the cache-line-size heuristic (Section "Cache Line Size
                   benchmarks"): strides from a pivot (surely below the line
                   size) to a MAX (surely above), array sizes around and above
                   the cache size. The reading:
      - per stride j and size index a, with the p50 latencies x, pivot row P =
        x[0] and MAX row M = x[J - 1]: dp = |x - P|, dm = |x - M|, similarity
        to MAX q = floor(2^32 dp / (dp + dm)) (0 when dp + dm = 0);
      - score_j = sum_a (a + 1) q_j(a), larger arrays weighing more (the
        weight a + 1), compared against W 2^32 with W = sum_a (a + 1);
      - j* = the first stride j >= 1 with score_j more than half the maximum
        (more similar to MAX than to the pivot); from j* on the score is the
        running maximum, so that an aliased stride that looks like the pivot
        again does not break the step;
      - the line size is a power of two: over the strides that are powers of
        two, in order, the largest increase of the adapted score between
        consecutive ones; the line size is the stride before it (at a stride
        up to the line size every line is still touched). Ties go to the
        smaller stride.
"""

from fractions import Fraction

import numpy as np

CHECK_EDGE_LOW = 1
CHECK_EDGE_HIGH = 2
CHECK_NO_CHANGE = 4
CHECK_DISTURBED = 8

CHECK_DTYPE = np.dtype([("flags", "<u4"), ("disturbed", "<u4"), ("lo", "<i4"), ("hi", "<i4"),
                        ("med_lo", "<u4"), ("med_hi", "<u4"), ("mad_lo", "<u4"), ("mad_hi", "<u4")])

LINE_INCONCLUSIVE = 1  # fewer than two power-of-two strides
LINE_NO_INCREASE = 2   # no score increase between power-of-two strides
LINE_NO_MAX_LIKE = 4   # no stride is more similar to MAX than to the pivot

LINE_DTYPE = np.dtype([("line", "<u4"), ("jstar", "<u4"), ("flags", "<u4"), ("pad", "<u4"), ("jump", "<f8")])


def lower_median(values) -> int:
    """x_(floor((n - 1) / 2)) of the values sorted ascending (n >= 1)."""
    s = sorted(int(v) for v in values)
    return s[(len(s) - 1) // 2]


def check_sweep(p50, cp: int, significant: bool, edge: int = 4, k: int = 5) -> np.ndarray:
    """Workflow step 3 for one sweep of K = len(p50) steps; returns one
    CHECK_DTYPE record (see the module docstring for the rule)."""
    v = [int(x) for x in p50]
    K = len(v)
    out = np.zeros((), CHECK_DTYPE)
    sides = [(0, cp), (cp, K)] if significant else [(0, K), (0, K)]
    meds, mads, disturbed = [], [], set()
    for a, b in sides:
        part = v[a:b]
        med = lower_median(part)
        dev = [abs(x - med) for x in part]
        mad = lower_median(dev)
        floor = max(1, med // 64)
        for i, d in enumerate(dev):
            if d > k * max(mad, floor):
                disturbed.add(a + i)
        meds.append(med)
        mads.append(mad)
    flags, lo, hi = 0, 0, K
    if not significant:
        flags |= CHECK_NO_CHANGE
        lo, hi = -K, 2 * K
    else:
        if cp < edge:
            flags |= CHECK_EDGE_LOW
            lo = -K
        if K - cp < edge:
            flags |= CHECK_EDGE_HIGH
            hi = 2 * K
    if disturbed:
        flags |= CHECK_DISTURBED
        lo = min(lo, -(K // 2))
        hi = max(hi, K + K // 2)
    out["flags"], out["disturbed"], out["lo"], out["hi"] = flags, len(disturbed), lo, hi
    out["med_lo"], out["med_hi"], out["mad_lo"], out["mad_hi"] = meds[0], meds[1], mads[0], mads[1]
    return out


def align_fraction(S: int, T: int) -> tuple[int, float, float]:
    """Nearest integer fraction T / k (k >= 1) of T to S, ties to the smaller k.
    Returns (k, T / k, |S k - T| / T), both ratios correctly rounded doubles.
    S, T >= 1 bytes."""
    S, T = int(S), int(T)
    best = None
    for k in range(max(1, T // S - 1), T // S + 3):
        d = abs(Fraction(S) - Fraction(T, k))
        if best is None or d < best[1]:
            best = (k, d)
    k = best[0]
    return k, float(Fraction(T, k)), float(Fraction(abs(S * k - T), T))


def line_size(x, strides) -> np.ndarray:
    """Cache-line-size heuristic for one experiment: x[j][a] the p50 latency at
    stride j (strides ascending, bytes) and array-size index a (ascending);
    returns one LINE_DTYPE record."""
    x = [[int(v) for v in row] for row in x]
    J, A = len(x), len(x[0])
    P, M = x[0], x[J - 1]
    W = A * (A + 1) // 2
    score = []
    for j in range(J):
        s = 0
        for a in range(A):
            dp, dm = abs(x[j][a] - P[a]), abs(x[j][a] - M[a])
            q = (dp << 32) // (dp + dm) if dp + dm else 0
            s += (a + 1) * q
        score.append(s)
    half = W << 31  # half of the largest score, W 2^32
    jstar = next((j for j in range(1, J) if score[j] > half), J)
    adapted = list(score)
    run = 0
    for j in range(jstar, J):
        run = max(run, score[j])
        adapted[j] = run
    cands = [j for j in range(J) if strides[j] > 0 and (int(strides[j]) & (int(strides[j]) - 1)) == 0]
    out = np.zeros((), LINE_DTYPE)
    out["jstar"] = jstar
    flags = 0 if jstar < J else LINE_NO_MAX_LIKE
    if len(cands) < 2:
        out["flags"] = flags | LINE_INCONCLUSIVE
        return out
    best_t, best_d = 0, None
    for t in range(len(cands) - 1):
        d = adapted[cands[t + 1]] - adapted[cands[t]]
        if best_d is None or d > best_d:
            best_t, best_d = t, d
    if best_d <= 0:
        flags |= LINE_NO_INCREASE
    out["line"] = int(strides[cands[best_t]])
    out["flags"] = flags
    out["jump"] = float(Fraction(best_d, W << 32))
    return out

"""CPU oracle for MT4G's K-S change-point detection (arXiv 2511.05958).

TEST INFRASTRUCTURE: a slow, plain restatement of the method that the GPU
path is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s ``cpu_baseline`` leg may import it. It shares no code with the
HIP path; the product never imports it.

The arithmetic lives in ``ks_oracle.c`` (exact integers, long double for the
p-value); this module is ctypes marshalling plus numpy views. Each function
cites the passage it restates:

* ``reduce``         eq. 2 (Section "Size benchmarks", workflow step 4)
* ``split_U``        the two-sample K-S statistic, D = max_x |F(x) - G(x)|,
                     lower side vs higher side of a candidate (Section
                     "Background", K-S test)
* ``scan_series``    every index a candidate, the most significant one chosen,
                     eq. 1 significance, p-value as confidence (workflow step 4)
* ``kolmogorov``     the asymptotic distribution behind eq. 1
* ``row_stats``      per-row latency statistics: the average, p50, p95 and
                     standard deviation (Section "Load Latency benchmarks"),
                     with minimum and maximum
* ``segment``        every level boundary of one sweep: the single-change
                     test applied again to both sides of each significant
                     split (project-defined extension of workflow steps 2-4)
* ``features``       per-row decile features of the learned proposal
                     (project-defined; minimum as in eq. 2)
* ``cnn``            the proposal network, forward / backward / Adam in FP64
                     with BF16 operand rounding (project-defined)
* ``check_sweep``, ``align_fraction``, ``line_size`` (in ``sweep.py``): the
                     workflow's outlier check and interval widening, the L2
                     segment alignment, the cache-line-size heuristic
"""

from __future__ import annotations

import ctypes
import math
import os
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "libks_oracle.so"

RESULT_DTYPE = np.dtype(
    [("cp", "<u4"), ("n", "<u4"), ("m", "<u4"), ("U", "<u4"), ("D", "<f8"), ("lambda", "<f8"),
     ("p", "<f8"), ("significant", "<u4"), ("status", "<u4")]
)
assert RESULT_DTYPE.itemsize == 48

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            from . import build as _b  # noqa: F401  (oracle/build.py)

            _b.build()
        lib = ctypes.CDLL(str(_LIB_PATH))
        vp = ctypes.c_void_p
        u32 = ctypes.c_uint32
        lib.oracle_reduce.argtypes = [vp, u32, u32, vp, vp, vp]
        lib.oracle_reduce.restype = None
        lib.oracle_split_U.argtypes = [vp, vp, u32, u32]
        lib.oracle_split_U.restype = ctypes.c_uint64
        lib.oracle_c_alpha.argtypes = [ctypes.c_double]
        lib.oracle_c_alpha.restype = ctypes.c_double
        lib.oracle_kolmogorov.argtypes = [ctypes.c_double]
        lib.oracle_kolmogorov.restype = ctypes.c_double
        lib.oracle_scan_series.argtypes = [vp, u32, u32, ctypes.c_double, vp, vp]
        lib.oracle_scan_batch.argtypes = [vp, vp, vp, vp, u32, ctypes.c_double, vp, vp, vp, ctypes.c_int]
        lib.oracle_features.argtypes = [vp, u32, u32, vp]
        lib.oracle_features.restype = None
        assert lib.oracle_result_size() == 48
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def reduce(r) -> tuple[int, list[int]]:
    """Eq. 2 squared: (global min, [Q_0..Q_{K-1}]) with Q_i = sum_j (r_ij - min)^2 exact."""
    r = _u32(r)
    K, N = r.shape
    lo = np.zeros(K, np.uint64)
    hi = np.zeros(K, np.uint64)
    mn = ctypes.c_uint32(0)
    _load().oracle_reduce(r.ctypes.data, K, N, ctypes.byref(mn), lo.ctypes.data, hi.ctypes.data)
    return int(mn.value), [(int(h) << 64) | int(l) for l, h in zip(lo, hi)]


def split_U(Q, c: int) -> int:
    """U_c = n m D_c for the split lower = Q[:c], higher = Q[c:]."""
    K = len(Q)
    lo = np.array([q & ((1 << 64) - 1) for q in Q], np.uint64)
    hi = np.array([q >> 64 for q in Q], np.uint64)
    return int(_load().oracle_split_U(lo.ctypes.data, hi.ctypes.data, K, c))


def c_alpha(alpha: float) -> float:
    """Eq. 1 constant: d_alpha^2 = c_alpha (n+m)/(n m), c_alpha = -1/2 ln(alpha/2)."""
    return float(_load().oracle_c_alpha(alpha))


def kolmogorov(lambda2: float) -> float:
    """Asymptotic Kolmogorov tail Q_KS(lambda) from lambda^2."""
    return float(_load().oracle_kolmogorov(lambda2))


def scan_series(r, alpha: float = 0.05, want_allU: bool = False):
    """Full detection on one [K][N] series. Returns a RESULT_DTYPE record (and U_c for c<K)."""
    r = _u32(r)
    K, N = r.shape
    res = np.zeros((), RESULT_DTYPE)
    allU = np.zeros(max(K, 1), np.uint32)
    _load().oracle_scan_series(r.ctypes.data, K, N, alpha, res.ctypes.data, allU.ctypes.data)
    return (res, allU) if want_allU else res


def features(r) -> np.ndarray:
    """Per-row decile features [K][9] (float32) of one [K][N] series."""
    r = _u32(r)
    K, N = r.shape
    out = np.zeros((K, 9), np.float32)
    _load().oracle_features(r.ctypes.data, K, N, out.ctypes.data)
    return out


def result_fields(K: int, c: int, U: int, alpha: float = 0.05) -> dict:
    """The reported fields of choice c with numerator U (same arithmetic as scan_series)."""
    n, m = c, K - c
    U2 = float(U * U)
    nmK = float(n * m * K)
    lam2 = U2 / nmK
    return {"cp": c, "n": n, "m": m, "U": U, "D": U / float(n * m), "lambda": float(np.sqrt(lam2)),
            "p": 1.0 if U == 0 else kolmogorov(lam2), "significant": int(U2 > c_alpha(alpha) * nmK)}


def refine(allU, K: int, proposal: int, confidence: float, w: int, tau: float, alpha: float = 0.05) -> dict:
    """Exact choice restricted to candidates within +-w of the proposal when confidence >= tau,
    over every candidate otherwise (fallback). allU[c] = U_c of the series (from scan_series).
    The choice is the most significant candidate of the range (largest U_c^2 / (c (K - c)),
    compared exactly), ties to the smaller c."""
    refined = bool(np.float32(confidence) >= np.float32(tau))
    if refined:
        lo, hi = max(1, proposal - w), min(K - 1, proposal + w)
        if lo > hi:  # a proposal outside 1..K-1 leaves an empty window: fall back
            refined, lo, hi = False, 1, K - 1
    else:
        lo, hi = 1, K - 1
    best = lo
    for c in range(lo + 1, hi + 1):
        if int(allU[c]) ** 2 * (best * (K - best)) > int(allU[best]) ** 2 * (c * (K - c)):
            best = c
    out = result_fields(K, best, int(allU[best]), alpha)
    out["refined"] = refined
    return out


ROW_STATS_DTYPE = np.dtype([("mean", "<f8"), ("std", "<f8"), ("min", "<u4"), ("p50", "<u4"), ("p95", "<u4"),
                            ("max", "<u4")])


def row_stats(r) -> np.ndarray:
    """Per-row latency statistics of a [K][N] series: the average as the main
    result, with p50, p95 and the standard deviation (Section "Load Latency
    benchmarks"), and the minimum and maximum. With exact integer sums
    s1 = sum r and s2 = sum r^2 of a row:
        mean = s1 / N, one correctly rounded division;
        std  = sqrt(float(N s2 - s1^2) / (N N)), the exact numerator rounded
               once to double, then double division and square root;
        p50, p95 = x_(floor(q (N - 1))) of the row sorted ascending, q = 0.5,
               0.95 (floor in exact integer arithmetic); min, max likewise.
    Plain Python integers, one row at a time."""
    r = _u32(r)
    K, N = r.shape
    out = np.zeros(K, ROW_STATS_DTYPE)
    for i in range(K):
        row = [int(v) for v in r[i]]
        s1 = sum(row)
        s2 = sum(v * v for v in row)
        srt = sorted(row)
        out[i]["mean"] = s1 / N
        out[i]["std"] = math.sqrt(float(N * s2 - s1 * s1) / float(N * N))
        out[i]["min"] = srt[0]
        out[i]["p50"] = srt[(N - 1) // 2]
        out[i]["p95"] = srt[(95 * (N - 1)) // 100]
        out[i]["max"] = srt[-1]
    return out


def segment(r, alpha: float = 0.05, max_levels: int = 0) -> list[dict]:
    """Binary segmentation of one [K][N] series into level boundaries.

    The paper's test finds one change point per application, and its workflow
    narrows the search interval until one boundary is isolated (workflow
    steps 2-4). To report every boundary of one sweep, the test is applied to a
    window of rows [a, b): the window is a series of its own (eq. 2 with the
    window's own global minimum, every index a candidate, eq. 1 significance).
    When the window's split c is significant, c is a boundary and both sides
    [a, c) and [c, b) are tested in turn. A window of fewer than 2 rows, or a
    non-significant one, ends its branch. Windows of depth d (0 = the whole
    series) are tested only while max_levels == 0 or d < max_levels.

    Returns one dict per boundary, sorted by position: cp (first row of the
    higher side, counted from row 0 of the series), the window's fields n, m,
    U, D, lambda, p (n = cp - a, m = b - cp) and its depth."""
    r = _u32(r)
    out = []
    stack = [(0, r.shape[0], 0)]
    while stack:
        a, b, depth = stack.pop()
        if b - a < 2 or (max_levels and depth >= max_levels):
            continue
        res = scan_series(r[a:b], alpha)
        if not res["significant"]:
            continue
        c = a + int(res["cp"])
        out.append({"cp": c, "n": int(res["n"]), "m": int(res["m"]), "U": int(res["U"]), "D": float(res["D"]),
                    "lambda": float(res["lambda"]), "p": float(res["p"]), "depth": depth})
        stack.append((a, c, depth + 1))
        stack.append((c, b, depth + 1))
    return sorted(out, key=lambda d: d["cp"])


def scan_batch(samples, offsets, Ks, Ns, alpha: float = 0.05, threads: int | None = None,
               want_allU: bool = False):
    """Detection on many series of one packed buffer; series t is samples[offsets[t]:][:K*N]."""
    samples = _u32(samples)
    offsets = np.ascontiguousarray(offsets, np.uint64)
    Ks = _u32(Ks)
    Ns = _u32(Ns)
    num = len(Ks)
    if threads is None:
        threads = os.cpu_count() or 1
    res = np.zeros(num, RESULT_DTYPE)
    if want_allU:
        aoff = np.zeros(num, np.uint64)
        if num:
            aoff[1:] = np.cumsum(Ks.astype(np.uint64))[:-1]
        allU = np.zeros(int(Ks.astype(np.uint64).sum()), np.uint32)
        _load().oracle_scan_batch(samples.ctypes.data, offsets.ctypes.data, Ks.ctypes.data, Ns.ctypes.data,
                                  num, alpha, res.ctypes.data, allU.ctypes.data, aoff.ctypes.data, threads)
        return res, allU, aoff
    _load().oracle_scan_batch(samples.ctypes.data, offsets.ctypes.data, Ks.ctypes.data, Ns.ctypes.data,
                              num, alpha, res.ctypes.data, None, None, threads)
    return res


from .sweep import (CHECK_DISTURBED, CHECK_DTYPE, CHECK_EDGE_HIGH, CHECK_EDGE_LOW, CHECK_NO_CHANGE,  # noqa: E402
                    LINE_DTYPE, LINE_INCONCLUSIVE, LINE_NO_INCREASE, LINE_NO_MAX_LIKE, align_fraction,
                    check_sweep, line_size, lower_median)

"""Pins of the oracle's per-row latency statistics (Section "Load Latency benchmarks":
the average as the main result, p50, p95 and the standard deviation beside it).

Independent references: numpy's percentiles with the 'lower' method (index
floor(q (N - 1)) of the sorted row), numpy min / max, numpy mean and population
standard deviation (float64, a few ulps apart from the exact-integer forms), and
closed forms of constant and two-valued rows.
"""

import math

import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("seed,K,N", [(0, 5, 1), (1, 4, 2), (2, 3, 7), (3, 6, 100), (4, 2, 1023), (5, 3, 4096)])
def test_row_stats_against_numpy(seed, K, N):
    rng = np.random.default_rng(seed)
    r = np.round(rng.lognormal(np.log(500), 0.3, (K, N)) * np.where(rng.random((K, N)) < 0.02, 4.0, 1.0))
    r = r.astype(np.uint32)
    st = O.row_stats(r)
    for i in range(K):
        row = r[i].astype(np.float64)
        assert st[i]["min"] == r[i].min() and st[i]["max"] == r[i].max()
        assert st[i]["p50"] == np.percentile(r[i], 50, method="lower")
        assert st[i]["p95"] == np.percentile(r[i], 95, method="lower")
        assert st[i]["mean"] == pytest.approx(row.mean(), rel=1e-15)
        assert st[i]["std"] == pytest.approx(row.std(ddof=0), rel=1e-12, abs=1e-12)


def test_row_stats_closed_forms():
    # constant row: std 0, every order statistic the value
    st = O.row_stats(np.full((1, 37), 4000000000, np.uint32))[0]
    assert (st["mean"], st["std"], st["min"], st["p50"], st["p95"], st["max"]) == (4e9, 0.0, 4e9, 4e9, 4e9, 4e9)
    # n_a copies of a and n_b of b: mean (n_a a + n_b b) / N, std |b - a| sqrt(n_a n_b) / N
    a, b, na, nb = 100, 700, 30, 70
    st = O.row_stats(np.array([[a] * na + [b] * nb], np.uint32))[0]
    N = na + nb
    assert st["mean"] == (na * a + nb * b) / N
    assert st["std"] == pytest.approx(abs(b - a) * math.sqrt(na * nb) / N, rel=1e-15)
    assert (st["p50"], st["p95"]) == (b, b)  # floor(0.5 * 99) = 49 >= 30
    st = O.row_stats(np.array([[b] * 96 + [a] * 4], np.uint32))[0]
    assert (st["min"], st["p50"], st["p95"], st["max"]) == (a, b, b, b)


def test_row_stats_large_values_are_exact():
    # sums beyond 2^64: the integer numerator of the variance is exact
    r = np.array([[0xFFFFFFFF, 0, 0xFFFFFFFF, 0]], np.uint32)
    st = O.row_stats(r)[0]
    assert st["mean"] == 0xFFFFFFFF / 2
    assert st["std"] == 0xFFFFFFFF / 2

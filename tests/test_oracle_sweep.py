"""Pins of the oracle's workflow checks (outlier check and widening, L2 segment
alignment, cache-line-size heuristic) against closed forms, brute force and
numpy's own order statistics."""

from fractions import Fraction

import numpy as np
import pytest

import oracle as O


def plateaus(levels, lengths):
    return np.concatenate([np.full(n, lv, np.int64) for lv, n in zip(levels, lengths)])


# ------------------------------------------------------------------ medians


@pytest.mark.parametrize("n", [1, 2, 3, 10, 257])
def test_lower_median_is_numpy_lower_percentile(n):
    rng = np.random.default_rng(n)
    v = rng.integers(0, 1000, n)
    assert O.lower_median(v) == int(np.percentile(v, 50, method="lower"))


# ------------------------------------------------------------------ workflow step 3


def test_clean_two_level_sweep_passes():
    p50 = plateaus([120, 300], [20, 30])
    c = O.check_sweep(p50, 20, True)
    assert int(c["flags"]) == 0 and int(c["disturbed"]) == 0
    assert (int(c["lo"]), int(c["hi"])) == (0, 50)
    assert (int(c["med_lo"]), int(c["med_hi"]), int(c["mad_lo"]), int(c["mad_hi"])) == (120, 300, 0, 0)


def test_one_disturbed_step_widens_both_ends():
    p50 = plateaus([120, 300], [20, 30])
    p50[7] = 360  # one step three times its level
    c = O.check_sweep(p50, 20, True)
    assert int(c["flags"]) == O.CHECK_DISTURBED and int(c["disturbed"]) == 1
    assert (int(c["lo"]), int(c["hi"])) == (-25, 75)


def test_disturbance_threshold_is_strict():
    # level 640: floor = 10, MAD = 0, threshold k * 10 = 50 cycles
    p50 = plateaus([640, 2000], [30, 30])
    p50[3] = 690
    assert int(O.check_sweep(p50, 30, True)["disturbed"]) == 0
    p50[3] = 691
    assert int(O.check_sweep(p50, 30, True)["disturbed"]) == 1
    p50[3] = 589  # below the level: |589 - 640| = 51
    assert int(O.check_sweep(p50, 30, True)["disturbed"]) == 1


def test_mad_matches_brute_force():
    rng = np.random.default_rng(3)
    for _ in range(50):
        K = int(rng.integers(4, 60))
        cp = int(rng.integers(1, K))
        p50 = rng.integers(100, 140, K) + np.where(np.arange(K) >= cp, 200, 0)
        c = O.check_sweep(p50, cp, True, k=2)
        for (a, b), med_f, mad_f in (((0, cp), "med_lo", "mad_lo"), ((cp, K), "med_hi", "mad_hi")):
            side = p50[a:b]
            med = int(np.percentile(side, 50, method="lower"))
            mad = int(np.percentile(np.abs(side - med), 50, method="lower"))
            assert (int(c[med_f]), int(c[mad_f])) == (med, mad)
        want = 0
        for a, b in ((0, cp), (cp, K)):
            side = p50[a:b]
            med = int(np.percentile(side, 50, method="lower"))
            mad = int(np.percentile(np.abs(side - med), 50, method="lower"))
            want += int(np.sum(np.abs(side - med) > 2 * max(mad, max(1, med // 64))))
        assert int(c["disturbed"]) == want


def test_change_close_to_a_boundary():
    p50 = plateaus([120, 300], [2, 40])
    c = O.check_sweep(p50, 2, True, edge=4)
    assert int(c["flags"]) == O.CHECK_EDGE_LOW and (int(c["lo"]), int(c["hi"])) == (-42, 42)
    p50 = plateaus([120, 300], [40, 3])
    c = O.check_sweep(p50, 40, True, edge=4)
    assert int(c["flags"]) == O.CHECK_EDGE_HIGH and (int(c["lo"]), int(c["hi"])) == (0, 86)
    c = O.check_sweep(p50, 40, True, edge=3)
    assert int(c["flags"]) == 0


def test_no_change_widens_by_the_interval_on_both_sides():
    p50 = np.full(33, 120)
    c = O.check_sweep(p50, 1, False)
    assert int(c["flags"]) == O.CHECK_NO_CHANGE
    assert (int(c["lo"]), int(c["hi"])) == (-33, 66)
    assert int(c["med_lo"]) == int(c["med_hi"]) == 120


# ------------------------------------------------------------------ L2 segment alignment


def test_exact_fractions():
    MiB = 1 << 20
    assert O.align_fraction(20 * MiB, 40 * MiB) == (2, 20.0 * MiB, 0.0)  # two 20 MB halves of a 40 MB L2
    assert O.align_fraction(4 * MiB, 32 * MiB) == (8, 4.0 * MiB, 0.0)
    assert O.align_fraction(64 * MiB, 32 * MiB)[0] == 1


def test_alignment_brute_force():
    rng = np.random.default_rng(5)
    for _ in range(300):
        T = int(rng.integers(1, 600))
        S = int(rng.integers(1, 700))
        dist = [abs(Fraction(S) - Fraction(T, k)) for k in range(1, T + 2)]
        k = int(np.argmin(dist)) + 1  # first minimum: the smaller k on ties
        got = O.align_fraction(S, T)
        assert got[0] == k, (S, T)
        assert got[2] == float(Fraction(abs(S * k - T), T))


# ------------------------------------------------------------------ cache line size


def step_profile(strides, line, A=12, hi=800, lo=300):
    """Strides up to the line size touch every line (pivot-like, misses above
    the cache size); larger strides skip lines (MAX-like)."""
    return np.array([[hi if s <= line else lo] * A for s in strides], np.int64)


@pytest.mark.parametrize("line", [32, 64, 128, 256])
def test_step_profile_gives_the_line_size(line):
    strides = [16 * (j + 1) for j in range(64)]  # pivot 16 B = fetch granularity / 2, step 16 B
    r = O.line_size(step_profile(strides, line), strides)
    assert int(r["line"]) == line and int(r["flags"]) == 0 and float(r["jump"]) == 1.0
    assert strides[int(r["jstar"])] == line + 16


def test_aliased_stride_does_not_move_the_answer():
    strides = [16, 32, 64, 128, 256, 512, 1024]
    P, M, A = 800, 300, 10
    x = np.array([[P] * A] * 7, np.int64)
    x[4:] = M                          # line 128: strides from 256 on skip lines
    x[4] = 800 - 0.6 * 500             # 256 only partly MAX-like ...
    x[5] = P                           # ... 512 aliases and looks like the pivot
    r = O.line_size(x, strides)
    assert int(r["line"]) == 128
    # without the running maximum from j* the largest increase would be 512 -> 1024
    score = [sum((a + 1) * ((abs(int(v) - P) << 32) // (abs(int(v) - P) + abs(int(v) - M))) for a, v in enumerate(row))
             for row in x]
    inc = [score[t + 1] - score[t] for t in range(6)]
    assert strides[int(np.argmax(inc))] == 512


def test_larger_arrays_weigh_more():
    strides = [16, 32, 64]
    A = 8
    x = np.array([[800] * A, [800] * 4 + [300] * 4, [300] * A], np.int64)
    assert int(O.line_size(x, strides)["jstar"]) == 1  # MAX-like on the larger half: score > 1/2
    x[1] = [300] * 4 + [800] * 4
    assert int(O.line_size(x, strides)["jstar"]) == 2


def test_similarity_midpoint_and_inconclusive():
    strides = [16, 32, 48]
    x = np.array([[800, 800], [550, 550], [300, 300]], np.int64)  # stride 32 halfway: q = 2^31
    r = O.line_size(x, strides)
    assert int(r["jstar"]) == 2  # exactly half is not "more similar to MAX"
    assert int(r["flags"]) & O.LINE_INCONCLUSIVE == 0 and int(r["line"]) == 16
    assert float(r["jump"]) == 0.5
    r = O.line_size(x, [16, 48, 80])
    assert int(r["flags"]) & O.LINE_INCONCLUSIVE

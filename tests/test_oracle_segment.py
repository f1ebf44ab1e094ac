"""Pins of the oracle's binary segmentation (every level boundary of a sweep).

Closed form: in a noise-free monotone staircase every row of a plateau has the
same eq. 2 value, so inside any window holding two or more whole plateaus the
split at a plateau boundary has D = 1 (every value of one side below every
value of the other) and lambda^2 = n m / K, while a window holding one
plateau is constant (U = 0, never significant). With plateaus of at least 4
rows, lambda^2 >= 4 * 4 / 8 = 2 > c_alpha(0.05) = 1.8444 for every window
with two plateaus or more, so the segmentation must return exactly the
plateau starts, each with D = 1.
"""

import numpy as np
import pytest

import oracle as O


def staircase(lengths, levels, N=16):
    rows = np.concatenate([np.full(n, lv, np.uint32) for n, lv in zip(lengths, levels)])
    return np.repeat(rows[:, None], N, axis=1)


def starts(lengths):
    return list(np.cumsum(lengths)[:-1])


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("order", ["ascending", "descending"])
def test_noise_free_staircase_finds_every_boundary(seed, order):
    rng = np.random.default_rng(seed)
    P = int(rng.integers(2, 9))
    lengths = rng.integers(4, 41, P)
    levels = np.sort(rng.choice(np.arange(50, 5000), P, replace=False))
    if order == "descending":
        levels = levels[::-1]
    r = staircase(lengths, levels)
    got = O.segment(r)
    assert [d["cp"] for d in got] == starts(lengths)
    for d in got:
        assert d["D"] == 1.0 and d["U"] == d["n"] * d["m"]


def test_constant_and_single_step():
    assert O.segment(np.full((50, 8), 7, np.uint32)) == []
    got = O.segment(staircase([20, 30], [100, 400]))
    assert [(d["cp"], d["n"], d["m"], d["depth"]) for d in got] == [(20, 20, 30, 0)]


def test_short_plateau_pair_is_not_significant():
    # two plateaus of 2 rows: lambda^2 = 2 * 2 / 4 = 1 < 1.8444, nothing is reported
    assert O.segment(staircase([2, 2], [100, 900])) == []


def test_max_levels_limits_depth_and_level_one_is_the_plain_scan():
    lengths = [6, 9, 12, 5, 8]
    r = staircase(lengths, [100, 200, 300, 400, 500])
    full = O.segment(r)
    assert [d["cp"] for d in full] == starts(lengths)
    one = O.segment(r, max_levels=1)
    top = O.scan_series(r)
    assert [(d["cp"], d["U"], d["depth"]) for d in one] == [(int(top["cp"]), int(top["U"]), 0)]
    two = O.segment(r, max_levels=2)
    assert all(d["depth"] <= 1 for d in two) and len(two) <= 3
    assert {d["cp"] for d in two} <= {d["cp"] for d in full}


def test_windows_nest():
    """Every boundary's window [cp - n, cp + m) is the whole series or one side of
    the window of a boundary one level up."""
    rng = np.random.default_rng(5)
    r = np.round(staircase([30, 20, 40, 25], [100, 300, 550, 850], N=64) *
                 np.exp(0.08 * rng.standard_normal((115, 64)))).astype(np.uint32)
    got = O.segment(r)
    assert len(got) >= 3
    K = r.shape[0]
    wins = {d["cp"]: (d["cp"] - d["n"], d["cp"] + d["m"], d["depth"]) for d in got}
    for cp, (a, b, depth) in wins.items():
        if depth == 0:
            assert (a, b) == (0, K)
        else:
            parents = [(pc, w) for pc, w in wins.items() if w[2] == depth - 1 and (a, b) in ((w[0], pc), (pc, w[1]))]
            assert len(parents) == 1, cp

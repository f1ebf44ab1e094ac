"""The seeded input generator: Philox known answers, reproducibility, recipe shapes."""

import math

import numpy as np

from paper_2511_05958_amd import synth as S


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 published with Random123 (Salmon et al., SC'11).
    assert S.philox4x32_10([0, 0, 0, 0], [0, 0]) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert S.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)
    assert S.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == (
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_generator_math_accuracy():
    for x in np.linspace(-20, 20, 401):
        assert abs(S.math_fn("exp", x) / math.exp(x) - 1) < 5e-16
    for x in np.exp(np.linspace(-25, 25, 401)):
        assert abs(S.math_fn("log", x) - math.log(x)) <= 5e-16 * max(1.0, abs(math.log(x)))
    for u in np.linspace(0, 0.9999, 401):
        assert abs(S.math_fn("cos2pi", u) - math.cos(2 * math.pi * u)) < 2e-15


def test_reproducible_and_batch_independent():
    b = S.make_batch(2, num_series=6)
    x1, x2 = S.fill_host(b, threads=1), S.fill_host(b, threads=3)
    assert np.array_equal(x1, x2)
    # a series regenerated alone (other batch composition) has the same samples
    sub = b.subset([4])
    xs = S.fill_host(sub)
    assert np.array_equal(S.series_view(xs, sub, 0), S.series_view(x1, b, 4))
    # the same ids requested from a later first_series give the same specs
    b2 = S.make_batch(2, num_series=2, first_series=4)
    assert np.array_equal(b2.specs[["K", "N", "nseg", "seg_start", "seg_level"]][0],
                          b.specs[["K", "N", "nseg", "seg_start", "seg_level"]][4])


def test_recipe_shapes():
    for r, (K, N) in {1: (64, 256), 2: (256, 1024), 5: (1024, 2048)}.items():
        b = S.make_batch(r, num_series=50)
        assert (b.specs["K"] == K).all() and (b.specs["N"] == N).all()
        assert (b.specs["offset"] % 64 == 0).all()
    b = S.make_batch(3, num_series=2000)
    K, N = b.specs["K"], b.specs["N"]
    assert K.min() >= 32 and K.max() <= 512 and N.min() >= 64 and N.max() <= 4096
    # log-uniform: the median sits near the geometric mean
    assert abs(np.log(np.median(K)) - 0.5 * (np.log(32) + np.log(512))) < 0.15
    assert abs(np.log(np.median(N)) - 0.5 * (np.log(64) + np.log(4096))) < 0.15
    # recipe 2: 1..4 plateaus of >= 8 rows each; recipe 5: 1..4 transitions
    b2 = S.make_batch(2, num_series=500)
    assert set(b2.specs["nplant"]) == {0, 1, 2, 3}
    for s in b2.specs:
        edges = list(s["seg_start"][: s["nseg"]]) + [256]
        assert min(np.diff(edges)) >= 8
    b5 = S.make_batch(5, num_series=200)
    assert set(b5.specs["nplant"]) == {1, 2, 3, 4}
    lv = b5.specs["seg_level"]
    for s in b5.specs:
        ratios = s["seg_level"][1: s["nseg"]] / s["seg_level"][: s["nseg"] - 1]
        assert ((ratios >= 1.05) & (ratios <= 1.2)).all()
    assert lv.shape[0] == 200


def test_noise_statistics():
    b = S.make_batch(5, num_series=2)
    x = S.fill_host(b)
    v = S.series_view(x, b, 0).astype(np.float64)
    L0 = b.specs[0]["seg_level"][0]
    row = v[0] / L0
    # 5% outliers in [1,5]; 10% Pareto(1, 2.5) multipliers (>= 1); the rest lognormal(0.08)
    assert 0.02 < np.mean(row > 1.5) < 0.12
    b1 = S.make_batch(1)
    y = S.series_view(S.fill_host(b1), b1, 0).astype(np.float64)
    lr = np.log(y[: b1.specs[0]["plant"][0]] / 120.0)
    assert abs(lr.std() - 0.05) < 0.005 and abs(lr.mean()) < 0.01

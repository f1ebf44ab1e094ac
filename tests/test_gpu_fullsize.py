"""Full-size batches in the launch configuration bench.py times (default plan).

Every series is checked against properties that hold at any size; a seeded
sample of series is copied back and recomputed one by one by the oracle
(bit-exact fields, p within 1e-12).
"""

import math

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from paper_2511_05958_amd import synth as S

pytestmark = pytest.mark.gpu


def run_full(recipe, sample_count, seed):
    import torch

    b = S.make_batch(recipe)
    n = b.num_series
    buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(b, buf.data_ptr(), b.total_elems)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    prm = P.ks_params_init(0.05)
    prm.max_K = int(d["K"].max())
    out = P.empty_results(n)
    with P.Context(0) as ctx:
        P.ks_scan_batch(ctx.handle, buf, P.to_device(d), n, prm, out)
        torch.cuda.synchronize()
    g = P.results_to_numpy(out)

    # properties of every series
    K = d["K"].astype(np.int64)
    cp, nn, mm, U = (g[f].astype(np.int64) for f in ("cp", "n", "m", "U"))
    assert (g["flags"] & (P.KS_BAD_SHAPE | P.KS_OUT_OF_RANGE) == 0).all()
    assert ((cp >= 1) & (cp < K) & (nn == cp) & (mm == K - cp)).all()
    assert (U <= nn * mm).all()
    assert np.array_equal(g["D"], U / (nn * mm))
    lam2 = (U * U).astype(np.float64) / (nn * mm * K).astype(np.float64)
    assert np.array_equal(g["lambda"], np.sqrt(lam2))
    sig = (U * U).astype(np.float64) > prm.c_alpha * (nn * mm * K).astype(np.float64)
    assert np.array_equal((g["flags"] & P.KS_SIGNIFICANT) != 0, sig)
    assert ((g["p"] >= 0) & (g["p"] <= 1)).all()

    # a seeded sample recomputed by the oracle
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(n, size=min(sample_count, n), replace=False))
    for t in pick:
        o0, k, nn_ = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"])
        r = buf[o0:o0 + k * nn_].cpu().numpy().view(np.uint32).reshape(k, nn_)
        o = O.scan_series(r)
        assert (g[t]["cp"], g[t]["U"], g[t]["n"], g[t]["m"]) == (o["cp"], o["U"], o["n"], o["m"]), t
        assert g[t]["D"] == o["D"] and g[t]["lambda"] == o["lambda"]
        assert bool(g[t]["flags"] & P.KS_SIGNIFICANT) == bool(o["significant"])
        assert g[t]["p"] == o["p"] or abs(g[t]["p"] - o["p"]) <= 1e-12 * abs(o["p"]), t
    del buf
    torch.cuda.empty_cache()
    return g


def test_recipe2_full_4096_series():
    g = run_full(2, 32, 2)
    assert len(g) == 4096


def test_recipe3_full_16384_uneven_series():
    g = run_full(3, 48, 3)
    assert len(g) == 16384


def test_recipe5_full_8192_series():
    g = run_full(5, 8, 5)
    assert len(g) == 8192
    assert math.isfinite(float(g["lambda"].max()))


@pytest.mark.parametrize("launch", [(P.KS_LAUNCH_ORDERED, 1 << 20, 1), (P.KS_LAUNCH_ORDERED, 1 << 20, 0),
                                    (P.KS_LAUNCH_PERSISTENT, 1 << 20, 1)],
                         ids=["ordered-graph", "ordered-direct", "persistent"])
def test_series_above_4gib_among_small_ones(launch):
    """A series of 64 rows x 2^24 samples (4 GiB of samples, more than a 32-bit
    byte count) among three small ones. The ordered plan must keep it one work
    item, so that its one-workgroup-per-series grid still covers every series.
    The big series is a noise-free step (rows < c0 at 120 cycles, the rest at
    121): its keys are Q = 0 below c0 and N above, so the closed form holds,
    c* = c0 and U* = c0 (K - c0); the small series are checked by the oracle."""
    import torch

    K, N, c0 = 64, 1 << 24, 40
    big = K * N
    b = S.make_batch(2, num_series=3, first_series=900)
    xs = S.fill_host(b)
    buf = torch.empty(big + len(xs), dtype=torch.int32, device="cuda")
    buf[:c0 * N].fill_(120)
    buf[c0 * N:big].fill_(121)
    buf[big:] = torch.from_numpy(xs.view(np.int32)).cuda()
    offs = np.concatenate([[0], big + b.specs["offset"].astype(np.int64)])
    d = P.make_desc(offs, np.concatenate([[K], b.specs["K"]]), np.concatenate([[N], b.specs["N"]]))
    prm = P.ks_params_init(0.05)
    prm.max_K = 256
    out = P.empty_results(4)
    out.fill_(0xA5)
    with P.Context(0) as ctx:
        P.ks_launch_set(ctx.handle, 256, 4, *launch)
        P.ks_scan_batch(ctx.handle, buf, P.to_device(d), 4, prm, out)
        torch.cuda.synchronize()
    g = P.results_to_numpy(out)
    assert (g[0]["cp"], g[0]["n"], g[0]["m"], g[0]["U"]) == (c0, c0, K - c0, c0 * (K - c0))
    assert g[0]["D"] == 1.0 and g[0]["flags"] & P.KS_SIGNIFICANT
    for t in range(1, 4):
        o0, k, n_ = int(d[t]["offset"]) - big, int(d[t]["K"]), int(d[t]["N"])
        o = O.scan_series(xs[o0:o0 + k * n_].reshape(k, n_))
        assert (g[t]["cp"], g[t]["U"], g[t]["n"], g[t]["m"]) == (o["cp"], o["U"], o["n"], o["m"]), t
        assert g[t]["flags"] == (P.KS_SIGNIFICANT if o["significant"] else 0), t
    del buf
    torch.cuda.empty_cache()


@pytest.mark.parametrize("recipe,how", [(5, "autotune"), (5, "persistent-16MiB-v2"), (3, "autotune")])
def test_full_batch_in_bench_launch_equals_default(recipe, how):
    """The full batch in the launch bench.py times: the plan the autotuner picks
    on this device (its default), or the one it picked for recipe 5 when the
    profiles were taken (persistent queue, 16 MiB splits, variant 2). Every
    series' result must equal, field by field, the library default plan's
    (another kernel and work split over the same samples), and a seeded sample
    is recomputed by the oracle."""
    import torch

    b = S.make_batch(recipe)
    n = b.num_series
    buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(b, buf.data_ptr(), b.total_elems)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    dd = P.to_device(d)
    prm = P.ks_params_init(0.05)
    prm.max_K = int(d["K"].max())
    out0, out1 = P.empty_results(n), P.empty_results(n)
    with P.Context(0) as ctx:
        P.ks_scan_batch(ctx.handle, buf, dd, n, prm, out0)
        if how == "autotune":
            P.ks_autotune(ctx.handle, buf, dd, n, prm, out1)
        else:
            P.ks_launch_set(ctx.handle, prm.max_K, n, P.KS_LAUNCH_PERSISTENT, 16 << 20, 0, variant=2)
        out1.fill_(0xA5)
        P.ks_scan_batch(ctx.handle, buf, dd, n, prm, out1)
        c = P.ks_launch_get(ctx.handle, prm.max_K, n)
        torch.cuda.synchronize()
    print("launch", how, c.mode, c.chunk_bytes, c.graph, c.variant, flush=True)
    g0, g1 = P.results_to_numpy(out0), P.results_to_numpy(out1)
    for f in ("cp", "n", "m", "U", "D", "lambda", "p", "flags"):
        assert np.array_equal(g0[f], g1[f]), f
    rng = np.random.default_rng(100 + recipe)
    for t in np.sort(rng.choice(n, size=4, replace=False)):
        o0, k, nn_ = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"])
        r = buf[o0:o0 + k * nn_].cpu().numpy().view(np.uint32).reshape(k, nn_)
        o = O.scan_series(r)
        assert (g1[t]["cp"], g1[t]["U"], g1[t]["n"], g1[t]["m"]) == (o["cp"], o["U"], o["n"], o["m"]), t
        assert g1[t]["D"] == o["D"] and g1[t]["lambda"] == o["lambda"]
        assert bool(g1[t]["flags"] & P.KS_SIGNIFICANT) == bool(o["significant"])
        assert g1[t]["p"] == o["p"] or abs(g1[t]["p"] - o["p"]) <= 1e-12 * abs(o["p"]), t
    del buf
    torch.cuda.empty_cache()

"""GPU parity of binary segmentation (ks_segment_batch) against the oracle's recursion.

Bar: the set of boundaries of every series equal to the oracle's, each with
bit-equal cp, n, m, U, D, lambda and depth, and p within 1e-12 relative.
"""

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from paper_2511_05958_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    c = P.Context(0)
    yield c
    c.close()


def run(ctx, x, d, max_K, max_levels=0, max_cp=None, x_dev=None):
    import torch

    n = len(d)
    max_cp = max_cp or max_K
    cps = torch.empty(n * max_cp * 48, dtype=torch.uint8, device="cuda")
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    prm = P.ks_params_init(0.05)
    prm.max_K = max_K
    P.ks_segment_batch(ctx.handle, P.to_device(x) if x_dev is None else x_dev, P.to_device(d), n, prm, max_levels,
                       max_cp, cps, counts)
    torch.cuda.synchronize()
    return cps.cpu().numpy().view(P.RESULT_DTYPE).reshape(n, max_cp), counts.cpu().numpy().view(np.uint32)


def series(x, d, t):
    o, K, N = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"])
    return x[o:o + K * N].reshape(K, N)


def check_series(got, count, ref, t):
    assert count == len(ref), (t, count, len(ref))
    for g, r in zip(got[:count], ref):
        assert (int(g["cp"]), int(g["n"]), int(g["m"]), int(g["U"]), int(g["pad"])) == \
            (r["cp"], r["n"], r["m"], r["U"], r["depth"]), t
        assert g["D"] == r["D"] and g["lambda"] == r["lambda"], t
        assert g["p"] == r["p"] or abs(g["p"] - r["p"]) <= 1e-12 * r["p"], t
        assert g["flags"] & P.KS_SIGNIFICANT


@pytest.mark.parametrize("recipe,num", [(1, 1), (2, 24), (3, 64), (5, 3)])
def test_segment_matches_oracle(ctx, recipe, num):
    b = S.make_batch(recipe, num_series=num)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    max_K = int(d["K"].max())
    cps, counts = run(ctx, x, d, max_K)
    total = 0
    for t in range(num):
        ref = O.segment(series(x, d, t))
        check_series(cps[t], int(counts[t]), ref, t)
        total += len(ref)
    assert total >= num  # the planted series do have boundaries


def test_segment_noise_free_staircases(ctx):
    rng = np.random.default_rng(11)
    parts, offs, Ks, want, off = [], [], [], [], 0
    for t in range(20):
        P_ = int(rng.integers(2, 9))
        lengths = rng.integers(4, 41, P_)
        levels = np.sort(rng.choice(np.arange(50, 5000), P_, replace=False))
        if t % 2:
            levels = levels[::-1]
        rows = np.concatenate([np.full(n, lv, np.uint32) for n, lv in zip(lengths, levels)])
        r = np.repeat(rows[:, None], 8, axis=1)
        offs.append(off)
        parts.append(r.ravel())
        off += r.size
        Ks.append(r.shape[0])
        want.append(list(np.cumsum(lengths)[:-1]))
    x = np.concatenate(parts)
    d = P.make_desc(offs, Ks, [8] * len(Ks))
    cps, counts = run(ctx, x, d, int(max(Ks)))
    for t in range(len(Ks)):
        assert [int(c) for c in cps[t]["cp"][:counts[t]]] == want[t], t
        assert np.all(cps[t]["D"][:counts[t]] == 1.0)


def test_levels_limit_and_level_one_is_the_plain_scan(ctx):
    import torch

    b = S.make_batch(2, num_series=16, first_series=40)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    cps, counts = run(ctx, x, d, 256, max_levels=1)
    out = P.empty_results(len(d))
    prm = P.ks_params_init(0.05)
    prm.max_K = 256
    P.ks_scan_batch(ctx.handle, P.to_device(x), P.to_device(d), len(d), prm, out)
    torch.cuda.synchronize()
    plain = P.results_to_numpy(out)
    for t in range(len(d)):
        sig = bool(plain[t]["flags"] & P.KS_SIGNIFICANT)
        assert counts[t] == int(sig), t
        if sig:
            assert (cps[t][0]["cp"], cps[t][0]["U"], cps[t][0]["pad"]) == (plain[t]["cp"], plain[t]["U"], 0)
    cps2, counts2 = run(ctx, x, d, 256, max_levels=2)
    for t in range(len(d)):
        ref = O.segment(series(x, d, t), max_levels=2)
        check_series(cps2[t], int(counts2[t]), ref, t)


@pytest.mark.parametrize("max_levels", [0, 1, 3, 4, 5, 6, 9, 13])
def test_deep_recursion_level_limits(ctx, max_levels):
    """Geometric staircases (plateaus of 256, 128, 64, ... rows) recurse about
    eight depths deep on one side; limits around the host's read-back chunks
    (depths 1-4, 5-12, 13-28) must cut exactly where the oracle's recursion does."""
    rng = np.random.default_rng(99)
    K, N = 512, 64
    ss = []
    for t in range(6):
        edges = [0] + [K - (K >> (j + 1)) for j in range(9)] + [K]
        lv = np.zeros(K)
        for j in range(len(edges) - 1):
            lv[edges[j]:edges[j + 1]] = 200 + 120 * j * (1 + 0.1 * t)
        r = np.round(lv[:, None] * rng.lognormal(0, 0.01 * (t % 3), (K, N)))
        ss.append(r.astype(np.uint32))
    b = S.make_batch(3, num_series=10, first_series=700)
    x3 = S.fill_host(b)
    parts, offs, Ks, Ns, off = [], [], [], [], 0
    for r in ss:
        offs.append(off)
        Ks.append(r.shape[0])
        Ns.append(r.shape[1])
        parts.append(r.ravel())
        off += r.size
    for t in range(10):
        o, k, n = int(b.specs["offset"][t]), int(b.specs["K"][t]), int(b.specs["N"][t])
        offs.append(off)
        Ks.append(k)
        Ns.append(n)
        parts.append(x3[o:o + k * n])
        off += k * n
    x = np.concatenate(parts)
    d = P.make_desc(offs, Ks, Ns)
    cps, counts = run(ctx, x, d, 512, max_levels=max_levels)
    deepest = 0
    for t in range(len(d)):
        ref = O.segment(series(x, d, t), max_levels=max_levels)
        check_series(cps[t], int(counts[t]), ref, t)
        deepest = max([deepest] + [r["depth"] for r in ref])
    if max_levels == 0:
        assert deepest >= 6  # the staircases recurse into the second read-back chunk (depths 5-12)


def test_truncation_and_malformed_descriptors(ctx):
    b = S.make_batch(2, num_series=8, first_series=7)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    refs = [O.segment(series(x, d, t)) for t in range(len(d))]
    cps, counts = run(ctx, x, d, 256, max_cp=1)
    for t in range(len(d)):
        assert counts[t] == len(refs[t])
        if refs[t]:
            assert int(cps[t][0]["cp"]) in {r["cp"] for r in refs[t]}
    bad = d.copy()
    bad[1]["K"] = 1                      # too few rows
    bad[3]["offset"] = len(x)            # past the samples
    bad[5]["K"] = 300                    # above max_K
    cps, counts = run(ctx, x, bad, 256)
    assert counts[1] == counts[3] == counts[5] == P.KS_SEGMENT_BAD
    for t in (0, 2, 4, 6, 7):
        check_series(cps[t], int(counts[t]), refs[t], t)


def test_segment_full_size_recipe2_sampled(ctx):
    """4096 x 256 x 1024 (the benchmark batch): 48 sampled series against the oracle, and
    for every series sorted, distinct boundaries whose windows nest."""
    import torch

    b = S.make_batch(2)
    n = b.num_series
    buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(b, buf.data_ptr(), b.total_elems)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    cps, counts = run(ctx, None, d, 256, max_cp=64, x_dev=buf)
    assert np.all(counts <= 64)
    for t in range(n):
        v = cps[t][:counts[t]]
        assert np.all(np.diff(v["cp"].astype(np.int64)) > 0)
        assert np.all((v["cp"] >= 1) & (v["cp"] <= 255))
        assert np.all(v["cp"] - v["n"] >= 0) and np.all(v["cp"] + v["m"] <= 256)
        assert np.all(v[v["pad"] == 0]["n"] + v[v["pad"] == 0]["m"] == 256)
    rng = np.random.default_rng(2)
    for t in rng.choice(n, 48, replace=False):
        o = int(d[t]["offset"])
        r = buf[o:o + 256 * 1024].cpu().numpy().view(np.uint32).reshape(256, 1024)
        check_series(cps[t], int(counts[t]), O.segment(r), int(t))


@pytest.mark.parametrize("recipe,count", [(3, 24), (5, 6)])
def test_segment_full_size_sampled(ctx, recipe, count):
    """The whole batch as the bench's segmentation leg runs it (64 boundaries
    at most per series; recipe 5: 64 GiB): every series' boundaries sorted,
    distinct and inside their series, a seeded sample against the oracle's
    recursion."""
    import torch

    b = S.make_batch(recipe)
    n = b.num_series
    buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(b, buf.data_ptr(), b.total_elems)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    cps, counts = run(ctx, None, d, int(d["K"].max()), max_cp=64, x_dev=buf)
    assert np.all(counts <= 64)
    Ks = d["K"].astype(np.int64)
    for t in range(n):
        v = cps[t][:counts[t]]
        cp = v["cp"].astype(np.int64)
        assert np.all(np.diff(cp) > 0) and np.all((cp >= 1) & (cp <= Ks[t] - 1)), t
        assert np.all(cp - v["n"] >= 0) and np.all(cp + v["m"] <= Ks[t]), t
    rng = np.random.default_rng(20 + recipe)
    for t in rng.choice(n, count, replace=False):
        o, k, nn_ = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"])
        r = buf[o:o + k * nn_].cpu().numpy().view(np.uint32).reshape(k, nn_)
        check_series(cps[t], int(counts[t]), O.segment(r), int(t))
    del buf
    torch.cuda.empty_cache()

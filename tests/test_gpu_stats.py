"""GPU parity of the per-row latency statistics (ks_stats_batch) against the oracle.

Bar: every field bit-equal (order statistics are integers; mean and std are the
same IEEE operations on exact integers on both sides).
"""

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from paper_2511_05958_amd import synth as S

from test_gpu_learned import _long_row_series, _select_stress_series

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(dev):
    c = P.Context(0)
    yield c
    c.close()


def gpu_stats(ctx, x, d, max_K, x_dev=None):
    import torch

    rows = int(d["K"].astype(np.int64).sum())
    out = torch.full((rows * 32,), 0xFF, dtype=torch.uint8, device="cuda")
    P.ks_stats_batch(ctx.handle, P.to_device(x) if x_dev is None else x_dev, P.to_device(d), len(d), max_K, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(P.ROW_STATS_DTYPE)


def same(g, r):
    return (g["min"] == r["min"]).all() and (g["p50"] == r["p50"]).all() and (g["p95"] == r["p95"]).all() and \
        (g["max"] == r["max"]).all() and np.array_equal(g["mean"], r["mean"]) and np.array_equal(g["std"], r["std"])


@pytest.mark.parametrize("recipe,num", [(1, 1), (2, 6), (3, 30), (5, 2)])
def test_stats_bit_exact(ctx, recipe, num):
    b = S.make_batch(recipe, num_series=num)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    g = gpu_stats(ctx, x, d, int(d["K"].max()))
    for t in range(num):
        o, K, N, a = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"]), int(d[t]["aux_offset"])
        assert same(g[a:a + K], O.row_stats(x[o:o + K * N].reshape(K, N))), t


def test_stats_every_class_alignment_and_range(ctx):
    ss = _select_stress_series()
    parts, offs, off = [], [], 0
    for r in ss:
        off += 2
        offs.append(off)
        parts.append(np.zeros(2, np.uint32))
        parts.append(r.ravel())
        off += r.size
    x = np.concatenate(parts)
    d = P.make_desc(offs, [r.shape[0] for r in ss], [r.shape[1] for r in ss])
    g = gpu_stats(ctx, x, d, 64)
    for t, r in enumerate(ss):
        a = int(d[t]["aux_offset"])
        assert same(g[a:a + r.shape[0]], O.row_stats(r)), (t, r.shape)


def test_stats_long_rows(ctx):
    """Rows longer than the register classes hold (streamed), every alignment,
    through the window, past it, over all 32 bits and with counts above 2^16."""
    ss = _long_row_series()
    parts, offs, off = [], [], 0
    for r in ss:
        off += 3
        offs.append(off)
        parts.append(np.zeros(3, np.uint32))
        parts.append(r.ravel())
        off += r.size
    x = np.concatenate(parts)
    d = P.make_desc(offs, [r.shape[0] for r in ss], [r.shape[1] for r in ss])
    g = gpu_stats(ctx, x, d, 64)
    for t, r in enumerate(ss):
        a = int(d[t]["aux_offset"])
        assert same(g[a:a + r.shape[0]], O.row_stats(r)), (t, r.shape)


def test_stats_malformed_series(ctx):
    b = S.make_batch(2, num_series=4, first_series=3)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    d[1]["N"] = 0                 # N < 1: a bad shape
    d[2]["offset"] = len(x)       # past the samples
    g = gpu_stats(ctx, x, d, 256)
    for t in (1, 2):
        a = int(d[t]["aux_offset"])
        assert np.isnan(g[a:a + 256]["mean"]).all() and np.isnan(g[a:a + 256]["std"]).all()
    for t in (0, 3):
        o, a = int(d[t]["offset"]), int(d[t]["aux_offset"])
        assert same(g[a:a + 256], O.row_stats(x[o:o + 256 * 1024].reshape(256, 1024)))


@pytest.mark.parametrize("recipe,count", [(2, 16), (3, 24), (5, 6)])
def test_stats_full_size_sampled(ctx, recipe, count):
    """The whole batch of a recipe (recipe 5: 64 GiB, the bench's statistics
    leg), every row checked against order and range properties, a seeded
    sample of series against the oracle."""
    import torch

    b = S.make_batch(recipe)
    buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(b, buf.data_ptr(), b.total_elems)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    g = gpu_stats(ctx, None, d, int(d["K"].max()), x_dev=buf)
    assert np.isfinite(g["mean"]).all() and (g["min"] <= g["p50"]).all() and (g["p50"] <= g["p95"]).all()
    assert (g["p95"] <= g["max"]).all() and (g["mean"] >= g["min"]).all() and (g["mean"] <= g["max"]).all()
    assert (g["std"] >= 0).all() and (g["std"] <= (g["max"] - g["min"]).astype(np.float64)).all()
    rng = np.random.default_rng(4 + recipe)
    for t in rng.choice(len(d), count, replace=False):
        o, a, k, n = int(d[t]["offset"]), int(d[t]["aux_offset"]), int(d[t]["K"]), int(d[t]["N"])
        r = buf[o:o + k * n].cpu().numpy().view(np.uint32).reshape(k, n)
        assert same(g[a:a + k], O.row_stats(r)), int(t)
    del buf
    torch.cuda.empty_cache()

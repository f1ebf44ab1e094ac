"""GPU parity of the workflow checks (include/ks_sweep.h) against the oracle.

The GPU chain is ks_scan_batch -> ks_stats_batch -> ks_check_batch / ks_line_batch
on the device; the oracle chain is scan_series / row_stats -> check_sweep /
line_size on the same samples (no oracle input comes from the GPU). Bar: every
field equal (integers exactly; the FP64 ratios are the same single divisions of
exact integers on both sides).
"""

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from paper_2511_05958_amd import synth as S

pytestmark = pytest.mark.gpu

CHECK_FIELDS = ("flags", "disturbed", "lo", "hi", "med_lo", "med_hi", "mad_lo", "mad_hi")


@pytest.fixture(scope="module")
def ctx(dev):
    c = P.Context(0)
    yield c
    c.close()


def gpu_check(ctx, x, d, max_K, edge=4, k=5, stats_rows=None):
    import torch

    n = len(d)
    xd, dd = P.to_device(x), P.to_device(d)
    res = P.empty_results(n)
    prm = P.ks_params_init(0.05)
    prm.max_K = max_K
    P.ks_scan_batch(ctx.handle, xd, dd, n, prm, res)
    rows = int((d["aux_offset"].astype(np.int64) + d["K"]).max())
    stats = torch.zeros(rows * 32, dtype=torch.uint8, device="cuda")
    P.ks_stats_batch(ctx.handle, xd, dd, n, max_K, stats)
    if stats_rows is not None:
        stats = stats[:stats_rows * 32]
    out = torch.full((n * 32,), 0xAB, dtype=torch.uint8, device="cuda")
    P.ks_check_batch(ctx.handle, dd, n, max_K, res, stats, out, edge, k)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(P.CHECK_DTYPE)


def oracle_check(x, d, t, edge=4, k=5):
    o, K, N = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"])
    r = x[o:o + K * N].reshape(K, N)
    res = O.scan_series(r)
    return O.check_sweep(O.row_stats(r)["p50"], int(res["cp"]), bool(res["significant"]), edge, k)


def assert_check(g, o, t):
    for f in CHECK_FIELDS:
        assert int(g[f]) == int(o[f]), (t, f, int(g[f]), int(o[f]))


@pytest.mark.parametrize("recipe,num", [(1, 1), (2, 16), (3, 60), (5, 2)])
def test_check_matches_oracle(ctx, recipe, num):
    b = S.make_batch(recipe, num_series=num)
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    g = gpu_check(ctx, x, d, int(d["K"].max()))
    for t in range(num):
        assert_check(g[t], oracle_check(x, d, t), t)


def sweeps_from_levels(rows_list, N=4):
    """Series whose rows are constant (every sample = the row's level), so the
    per-step p50 is exactly the level."""
    parts, offs, Ks, off = [], [], [], 0
    for rows in rows_list:
        r = np.repeat(np.asarray(rows, np.uint32)[:, None], N, axis=1)
        offs.append(off)
        Ks.append(len(rows))
        parts.append(r.ravel())
        off += r.size
    return np.concatenate(parts), P.make_desc(offs, Ks, [N] * len(Ks))


def test_check_constructed_sweeps(ctx):
    rng = np.random.default_rng(21)
    sweeps = []
    for t in range(40):
        K = int(rng.integers(8, 300))
        c0 = int(rng.integers(1, K))
        lv = np.where(np.arange(K) < c0, 120, 300) + rng.integers(0, 4, K)
        for _ in range(int(rng.integers(0, 3))):  # disturbed steps
            lv[int(rng.integers(0, K))] *= int(rng.integers(2, 4))
        sweeps.append(lv)
    sweeps.append(np.full(50, 200))                              # no change
    sweeps.append(np.r_[np.full(2, 120), np.full(60, 300)])      # close to the low end
    sweeps.append(np.r_[np.full(60, 120), np.full(3, 300)])      # close to the high end
    sweeps.append(np.r_[np.full(30, 640), np.full(30, 2000)])
    sweeps[-1][3] = 691                                          # just past k * floor
    x, d = sweeps_from_levels(sweeps)
    for edge, k in ((4, 5), (1, 1), (8, 3)):
        g = gpu_check(ctx, x, d, int(d["K"].max()), edge=edge, k=k)
        for t in range(len(d)):
            assert_check(g[t], oracle_check(x, d, t, edge, k), t)
    g = gpu_check(ctx, x, d, int(d["K"].max()))
    assert int(g[-4]["flags"]) == P.KS_CHECK_NO_CHANGE
    assert int(g[-3]["flags"]) & P.KS_CHECK_EDGE_LOW and int(g[-2]["flags"]) & P.KS_CHECK_EDGE_HIGH
    assert int(g[-1]["disturbed"]) == 1


@pytest.mark.parametrize("recipe,count", [(2, 24), (3, 24), (5, 8)])
def test_check_full_size_sampled(ctx, recipe, count):
    """The whole batch as the bench's check leg runs it (recipe 5: 8192 sweeps of
    1024 steps, 64 GiB): no sweep flagged invalid, a seeded sample of sweeps
    against the oracle's scan, per-step p50 and check."""
    import torch

    b = S.make_batch(recipe)
    n = b.num_series
    buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
    S.fill_device(b, buf.data_ptr(), b.total_elems)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    dd = P.to_device(d)
    max_K = int(d["K"].max())
    rows = int(d["K"].astype(np.int64).sum())
    res = P.empty_results(n)
    prm = P.ks_params_init(0.05)
    prm.max_K = max_K
    P.ks_scan_batch(ctx.handle, buf, dd, n, prm, res)
    stats = torch.zeros(rows * 32, dtype=torch.uint8, device="cuda")
    P.ks_stats_batch(ctx.handle, buf, dd, n, max_K, stats)
    out = torch.zeros(n * 32, dtype=torch.uint8, device="cuda")
    P.ks_check_batch(ctx.handle, dd, n, max_K, res, stats, out)
    torch.cuda.synchronize()
    g = out.cpu().numpy().view(P.CHECK_DTYPE)
    assert not np.any(g["flags"] & P.KS_CHECK_INVALID)
    rng = np.random.default_rng(4 + recipe)
    for t in rng.choice(n, count, replace=False):
        o, k, nn_ = int(d[t]["offset"]), int(d[t]["K"]), int(d[t]["N"])
        r = buf[o:o + k * nn_].cpu().numpy().view(np.uint32).reshape(k, nn_)
        res_o = O.scan_series(r)
        assert_check(g[t], O.check_sweep(O.row_stats(r)["p50"], int(res_o["cp"]), bool(res_o["significant"])), t)
    del buf
    torch.cuda.empty_cache()


def test_check_invalid_inputs(ctx):
    x, d = sweeps_from_levels([np.r_[np.full(10, 100), np.full(10, 400)]] * 3)
    g = gpu_check(ctx, x, d, 20)
    assert not np.any(g["flags"] & P.KS_CHECK_INVALID)
    bad = d.copy()
    bad[1]["K"] = 1                       # flagged by the scan
    g = gpu_check(ctx, x, bad, 20)
    assert int(g[1]["flags"]) == P.KS_CHECK_INVALID and int(g[0]["flags"]) & P.KS_CHECK_INVALID == 0
    g = gpu_check(ctx, x, d, 20, stats_rows=45)  # the third sweep's steps end past the rows given
    assert int(g[2]["flags"]) == P.KS_CHECK_INVALID and int(g[1]["flags"]) & P.KS_CHECK_INVALID == 0
    with pytest.raises(P.KsError):
        gpu_check(ctx, x, d, 20, edge=0)


# ------------------------------------------------------------------ L2 alignment


def test_align_matches_oracle(dev):
    import torch

    rng = np.random.default_rng(8)
    MiB = 1 << 20
    S_ = [20 * MiB, 19 * MiB + 512 * 1024, 5, 12, 40 * MiB, 1, 7 * MiB] + list(rng.integers(1, 1 << 40, 500))
    T_ = [40 * MiB, 40 * MiB, 12, 12, 40 * MiB, 1, 96 * MiB] + list(rng.integers(1, 1 << 40, 500))
    S_ += list(rng.integers(1, 5000, 200))
    T_ += list(rng.integers(1, 1 << 30, 200))
    S_ += [0, 1, 1 << 50, 3]
    T_ += [10, 1 << 50, 10, 1 << 45]     # out of range: S = 0, T >= 2^50, S >= 2^50, T / S >= 2^32 - 16
    n = len(S_)
    Sd = torch.tensor(np.array(S_, np.uint64).view(np.int64), device="cuda")
    Td = torch.tensor(np.array(T_, np.uint64).view(np.int64), device="cuda")
    seg = torch.empty(n, dtype=torch.int32, device="cuda")
    al = torch.empty(n, dtype=torch.float64, device="cuda")
    di = torch.empty(n, dtype=torch.float64, device="cuda")
    P.ks_align_batch(Sd, Td, n, seg, al, di)
    torch.cuda.synchronize()
    seg, al, di = seg.cpu().numpy().view(np.uint32), al.cpu().numpy(), di.cpu().numpy()
    for i in range(n - 4):
        k, a, dist = O.align_fraction(int(S_[i]), int(T_[i]))
        assert (int(seg[i]), al[i], di[i]) == (k, a, dist), (i, S_[i], T_[i])
    assert (seg[:7] == [2, 2, 2, 1, 1, 1, 14]).all() and di[0] == 0.0 and di[3] == 0.0
    assert (seg[-4:] == 0).all() and np.isnan(al[-4:]).all() and np.isnan(di[-4:]).all()


# ------------------------------------------------------------------ cache line size


def line_experiments(rng, n, J, A, N, strides, kinds):
    """Latency samples of n experiments (J strides x A sizes x N samples each):
    strides up to the line miss above the cache size, larger ones skip lines."""
    exps, lines = [], []
    for e in range(n):
        kind = kinds[e % len(kinds)]
        pow2 = [s for s in strides if s & (s - 1) == 0][:-1]
        L = int(pow2[int(rng.integers(0, len(pow2)))])
        hi, lo = int(rng.integers(500, 900)), int(rng.integers(200, 400))
        lat = np.empty((J, A), np.int64)
        for j, s in enumerate(strides):
            frac = np.linspace(0.3, 1.0, A)                       # misses grow with the array size
            miss = frac if s <= L else frac * (L / s)              # skipped lines: a smaller footprint
            lat[j] = lo + (hi - lo) * miss
        if kind == "alias":
            big = [j for j, s in enumerate(strides) if s > 2 * L and j < J - 1]
            if big:
                lat[big[int(rng.integers(0, len(big)))]] = lat[0]  # one stride aliases like the pivot
        elif kind == "random":
            lat = rng.integers(100, 1000, (J, A))
        noise = rng.integers(0, 9, (J, A, N)) if kind != "flat" else np.zeros((J, A, N), np.int64)
        exps.append((lat[:, :, None] + noise).astype(np.uint32).reshape(J * A, N))
        lines.append(L)
    return exps, lines


def gpu_line(ctx, exps, J, strides, K_override=None):
    import torch

    N = exps[0].shape[1]
    x = np.concatenate([e.ravel() for e in exps])
    Ks = [e.shape[0] for e in exps]
    offs = np.cumsum([0] + [e.size for e in exps[:-1]])
    d = P.make_desc(offs, Ks, [N] * len(exps))
    rows = int(sum(Ks))
    if K_override:
        for t, K in K_override.items():
            d[t]["K"] = K
    dd = P.to_device(d)
    stats = torch.zeros(rows * 32, dtype=torch.uint8, device="cuda")
    P.ks_stats_batch(ctx.handle, P.to_device(x), dd, len(d), int(d["K"].max()), stats)
    st = torch.tensor(np.array(strides, np.uint32).view(np.int32), device="cuda")
    out = torch.full((len(d) * 24,), 0xCD, dtype=torch.uint8, device="cuda")
    P.ks_line_batch(ctx.handle, dd, len(d), stats, J, st, out)
    torch.cuda.synchronize()
    return out.cpu().numpy().view(P.LINE_DTYPE)


def assert_line(g, o, e):
    assert (int(g["line"]), int(g["jstar"]), int(g["flags"])) == (int(o["line"]), int(o["jstar"]), int(o["flags"])), e
    assert g["jump"] == o["jump"], e


@pytest.mark.parametrize("J,A,N", [(16, 32, 64), (2, 1, 16), (64, 8, 16), (8, 256, 16), (40, 5, 33)])
def test_line_matches_oracle(ctx, J, A, N):
    rng = np.random.default_rng(J * 1000 + A)
    strides = [16 * (j + 1) for j in range(J)]
    exps, lines = line_experiments(rng, 24, J, A, N, strides, ["clean", "alias", "random", "flat"])
    g = gpu_line(ctx, exps, J, strides)
    for e, x in enumerate(exps):
        p50 = O.row_stats(x)["p50"].reshape(J, A)
        assert_line(g[e], O.line_size(p50, strides), e)
    if J >= 8:  # the clean and aliased profiles are found
        for e in range(0, 24, 4):
            assert int(g[e]["line"]) == lines[e], e


def test_line_power_of_two_strides_and_invalid(ctx):
    rng = np.random.default_rng(77)
    J, A, N = 7, 12, 16
    strides = [16, 32, 64, 128, 256, 512, 1024]
    exps, _ = line_experiments(rng, 12, J, A, N, strides, ["clean", "alias", "random"])
    g = gpu_line(ctx, exps, J, strides, K_override={5: J * A - 1})
    for e, x in enumerate(exps):
        if e == 5:
            assert int(g[e]["flags"]) == P.KS_LINE_INVALID
            continue
        assert_line(g[e], O.line_size(O.row_stats(x)["p50"].reshape(J, A), strides), e)
    g = gpu_line(ctx, exps[:3], J, [16, 48, 80, 112, 144, 176, 208])  # one power of two: inconclusive
    assert all(int(r["flags"]) & P.KS_LINE_INCONCLUSIVE for r in g)

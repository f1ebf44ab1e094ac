"""GPU parity of ks_scan_batch against the CPU oracle, through the C ABI.

Bar: change point, side sizes, D numerator U, significance flag and every
U_c bit-exact; D and lambda bit-exact (single IEEE operations on exact
integers on both sides); p within 1e-12 relative.
"""

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from paper_2511_05958_amd import synth as S

pytestmark = pytest.mark.gpu

P_RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx(dev):
    c = P.Context(0)
    yield c
    c.close()


DEFAULT_LAUNCH = (P.KS_LAUNCH_ORDERED, 1 << 20, 1)
LAUNCHES = [(P.KS_LAUNCH_GRID, 1 << 20, 0), (P.KS_LAUNCH_ORDERED, 1 << 20, 1), (P.KS_LAUNCH_ORDERED, 1 << 20, 0),
            (P.KS_LAUNCH_PERSISTENT, 1 << 20, 1), (P.KS_LAUNCH_PERSISTENT, 64 << 10, 1),
            (P.KS_LAUNCH_PERSISTENT, 16 << 10, 0)]
LAUNCH_IDS = ["grid", "ordered-graph", "ordered-direct", "persistent", "split64k-graph", "split16k-direct"]


def run_gpu(ctx, samples, desc, alpha=0.05, max_K=0, allU_len=None, num_samples=None, launch=None, variant=0):
    import torch

    n = len(desc)
    prm = P.ks_params_init(alpha)
    prm.max_K = max_K
    P.ks_launch_set(ctx.handle, max_K, n, *(launch or DEFAULT_LAUNCH), variant=variant)
    s_d = P.to_device(samples) if len(samples) else torch.zeros(1, dtype=torch.int32, device="cuda")
    d_d = P.to_device(desc) if n else torch.zeros(24, dtype=torch.uint8, device="cuda")
    out = P.empty_results(max(n, 1))
    if allU_len is None:
        allU_len = int(np.sum(desc["K"].astype(np.int64))) if n else 0
    allU = torch.full((max(allU_len, 1),), -1, dtype=torch.int32, device="cuda")
    P.ks_scan_batch(ctx.handle, s_d, d_d, n, prm, out, allU[:allU_len] if allU_len else None,
                    num_samples=num_samples if num_samples is not None else len(samples))
    torch.cuda.synchronize()
    return P.results_to_numpy(out)[:n], allU.cpu().numpy().view(np.uint32)[:allU_len]


def oracle_batch(samples, desc, alpha=0.05):
    return O.scan_batch(samples, desc["offset"], desc["K"], desc["N"], alpha=alpha, want_allU=True)


def assert_parity(g, gU, o, oU, desc):
    assert len(g) == len(o)
    ok = o["status"] == 0
    for f in ("cp", "n", "m", "U"):
        bad = np.nonzero(g[f][ok] != o[f][ok])[0]
        assert bad.size == 0, f"{f} differs at series {np.nonzero(ok)[0][bad[:5]]}"
    assert np.array_equal(g["flags"][ok] & P.KS_SIGNIFICANT, o["significant"][ok])
    assert np.array_equal(g["D"][ok], o["D"][ok])
    assert np.array_equal(g["lambda"][ok], o["lambda"][ok])
    rel = np.abs(g["p"][ok] - o["p"][ok]) / np.maximum(np.abs(o["p"][ok]), 1e-300)
    assert np.all((rel <= P_RTOL) | (g["p"][ok] == o["p"][ok])), rel.max()
    assert np.array_equal(gU, oU)


def batch_arrays(b):
    x = S.fill_host(b)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    return x, d


@pytest.mark.parametrize("launch", LAUNCHES, ids=LAUNCH_IDS)
@pytest.mark.parametrize("recipe,num", [(1, 1), (2, 48), (3, 160), (5, 6)])
def test_parity_recipes(ctx, recipe, num, launch):
    b = S.make_batch(recipe, num_series=num)
    x, d = batch_arrays(b)
    max_K = int(d["K"].max())
    g, gU = run_gpu(ctx, x, d, max_K=max_K, launch=launch)
    o, oU, _ = oracle_batch(x, d)
    assert_parity(g, gU, o, oU, d)


VARIANT_LAUNCHES = [(P.KS_LAUNCH_GRID, 1 << 20, 0), (P.KS_LAUNCH_ORDERED, 1 << 20, 1),
                    (P.KS_LAUNCH_PERSISTENT, 64 << 10, 0)]


@pytest.fixture(scope="module")
def variant_batch():
    """Recipes 1, 2, 3 and 5 plus a K = 2048 staircase with ties: every K
    class, long and short walks, several sort passes; with the oracle's
    results (computed once for all variants)."""
    rng = np.random.default_rng(17)
    series = []
    for recipe, num, first in [(1, 2, 3), (2, 8, 70), (3, 40, 900), (5, 2, 30)]:
        b = S.make_batch(recipe, num_series=num, first_series=first)
        x, d = batch_arrays(b)
        series += [x[int(o):int(o) + int(K) * int(N)].reshape(int(K), int(N)) for o, K, N in
                   zip(d["offset"], d["K"], d["N"])]
    series.append(np.repeat((np.arange(2048) // 300 * 11 + 100)[:, None], 5, axis=1).astype(np.uint32)
                  + rng.integers(0, 3, (2048, 5), dtype=np.uint32))
    offs, off, xs = [], 0, []
    for r in series:
        offs.append(off)
        xs.append(r.ravel())
        off += r.size
    x = np.concatenate(xs)
    d = P.make_desc(offs, [r.shape[0] for r in series], [r.shape[1] for r in series])
    o, oU, _ = oracle_batch(x, d)
    return x, d, o, oU


@pytest.mark.parametrize("variant", range(P.KS_SCAN_VARIANTS))
@pytest.mark.parametrize("launch", VARIANT_LAUNCHES, ids=["grid", "ordered-graph", "split64k-direct"])
def test_parity_kernel_variants(ctx, variant_batch, variant, launch):
    """Every scan-kernel variant the autotuner chooses among (tile = workgroup
    size, radix digit bits of the key sort, walk window) in the grid, ordered
    and split persistent plans: bit-exact with the oracle."""
    x, d, o, oU = variant_batch
    g, gU = run_gpu(ctx, x, d, max_K=2048, launch=launch, variant=variant)
    assert_parity(g, gU, o, oU, d)
    assert P.ks_launch_get(ctx.handle, 2048, len(d)).variant == variant


def test_graph_replay_with_new_buffers(ctx):
    # same shape (so the cached graph is reused and its arguments updated), different data
    for first in (0, 40, 80):
        b = S.make_batch(3, num_series=40, first_series=first)
        x, d = batch_arrays(b)
        for ln in (LAUNCHES[1], LAUNCHES[4]):
            g, gU = run_gpu(ctx, x, d, max_K=512, launch=ln)
            o, oU, _ = oracle_batch(x, d)
            assert_parity(g, gU, o, oU, d)


def test_autotune_then_scan(ctx):
    import torch

    b = S.make_batch(3, num_series=64, first_series=1000)
    x, d = batch_arrays(b)
    prm = P.ks_params_init(0.05)
    prm.max_K = 512
    s_d, d_d, out = P.to_device(x), P.to_device(d), P.empty_results(len(d))
    best, ms = P.ks_autotune(ctx.handle, s_d, d_d, len(d), prm, out)
    assert best.mode in (0, 1, 2) and 0 <= best.variant < P.KS_SCAN_VARIANTS and ms > 0
    got = P.ks_launch_get(ctx.handle, 512, len(d))
    assert (got.mode, got.chunk_bytes, got.graph, got.variant) == (best.mode, best.chunk_bytes, best.graph,
                                                                    best.variant)
    torch.cuda.synchronize()
    o, oU, _ = oracle_batch(x, d)
    g = P.results_to_numpy(out)
    assert np.array_equal(g["cp"], o["cp"]) and np.array_equal(g["U"], o["U"])


def test_parity_recipe1_many_draws(ctx):
    b = S.make_batch(1, num_series=256, seed=S.seed_for(1) ^ 0x1234)
    x, d = batch_arrays(b)
    g, gU = run_gpu(ctx, x, d, max_K=64)
    o, oU, _ = oracle_batch(x, d)
    assert_parity(g, gU, o, oU, d)


@pytest.mark.parametrize("launch", [LAUNCHES[0], LAUNCHES[1], LAUNCHES[5]], ids=["grid", "ordered", "split16k-direct"])
def test_parity_all_K_variants_and_alpha(ctx, launch):
    # one launch per LDS variant, K at the top of each class; N on both sides of
    # the row-group limits (a 16- or 32-lane group per row up to 256 / 512
    # samples), series starts shifted by 0-3 elements off 16-byte alignment
    rng = np.random.default_rng(7)
    for K in (64, 128, 256, 512, 1024, 2048):
        Ns = [1, 3, 64, 255, 256, 257, 511, 512, 513]
        parts, offs, off = [], [], 0
        for j, N in enumerate(Ns):
            shift = j % 4
            parts.append(np.zeros(shift, np.uint32))
            r = rng.integers(100, 140, (K, N), dtype=np.uint32)
            r[K // 3:] += 25
            parts.append(r.ravel())
            pad = (-(shift + r.size)) % 64
            parts.append(np.zeros(pad, np.uint32))
            offs.append(off + shift)
            off += shift + r.size + pad
        x = np.concatenate(parts)
        d = P.make_desc(offs, [K] * len(Ns), Ns)
        for alpha in (0.05, 0.001):
            g, gU = run_gpu(ctx, x, d, alpha=alpha, max_K=K, launch=launch)
            o, oU, _ = oracle_batch(x, d, alpha=alpha)
            assert_parity(g, gU, o, oU, d)


@pytest.mark.parametrize("launch", LAUNCHES, ids=LAUNCH_IDS)
def test_edge_cases(ctx, launch):
    rng = np.random.default_rng(11)
    series = []
    series.append(np.array([[5], [9]], np.uint32))                       # K=2, N=1
    series.append(np.full((17, 5), 77, np.uint32))                       # all equal: U = 0
    series.append(rng.integers(0, 2, (300, 7), dtype=np.uint32) + 100)   # heavy ties
    big = np.full((40, 9), 0xFFFFFFFF, np.uint32)                        # Q beyond 64 bits
    big[:, 0] = 0
    big[20:, 1] = 5
    series.append(big)
    q = rng.integers(0, 4, (129, 1), dtype=np.uint32) * 1000             # quantized, N=1
    series.append(q)
    step = np.full((64, 33), 120, np.uint32)
    step[40:] = 320                                                      # noise-free, odd N
    series.append(step)
    parts, offs, off = [], [], 0
    for r in series:
        # unaligned offsets on purpose (exercise the dword path)
        offs.append(off + 1)
        parts.append(np.zeros(1, np.uint32))
        parts.append(r.ravel())
        off += 1 + r.size
    x = np.concatenate(parts)
    d = P.make_desc(offs, [r.shape[0] for r in series], [r.shape[1] for r in series])
    g, gU = run_gpu(ctx, x, d, max_K=512, launch=launch)
    o, oU, _ = oracle_batch(x, d)
    assert_parity(g, gU, o, oU, d)
    assert g[1]["cp"] == 1 and g[1]["U"] == 0 and g[1]["p"] == 1.0
    assert g[5]["cp"] == 40


@pytest.mark.parametrize("launch", LAUNCHES, ids=LAUNCH_IDS)
def test_bad_shapes_and_ranges(ctx, launch):
    x = np.arange(1000, dtype=np.uint32)
    d = P.make_desc([0, 0, 0, 0, 990, 2**40, 0], [1, 2, 600, 10, 2, 2, 2], [5, 0, 1, 10, 6, 1, 1])
    g, gU = run_gpu(ctx, x, d, max_K=512, launch=launch)
    err = g["flags"] & (P.KS_BAD_SHAPE | P.KS_OUT_OF_RANGE)
    assert list(err[:4]) == [P.KS_BAD_SHAPE, P.KS_BAD_SHAPE, P.KS_BAD_SHAPE, 0]
    assert list(err[4:6]) == [P.KS_OUT_OF_RANGE, P.KS_OUT_OF_RANGE]
    assert g[3]["flags"] & P.KS_SIGNIFICANT  # 0..99 in rows of 10: a ramp
    assert (g["cp"][[0, 1, 2, 4, 5]] == 0).all()
    assert g[6]["cp"] == 1 and g[6]["flags"] & P.KS_BAD_SHAPE == 0


def test_allU_bounds_and_empty_batch(ctx):
    b = S.make_batch(2, num_series=3)
    x, d = batch_arrays(b)
    # room for the first two series only: the third writes nothing
    g, gU = run_gpu(ctx, x, d, max_K=256, allU_len=512 + 100)
    o, oU, _ = oracle_batch(x, d)
    assert np.array_equal(gU[:512], oU[:512])
    assert (gU[512:] == 0xFFFFFFFF).all()
    assert np.array_equal(g["U"], o["U"])
    g0, _ = run_gpu(ctx, x, d[:0], max_K=256)
    assert len(g0) == 0


def test_host_validation(ctx):
    import torch

    x = torch.zeros(64, dtype=torch.int32, device="cuda")
    d = P.to_device(P.make_desc([0], [2], [2]))
    out = P.empty_results(1)
    prm = P.ks_params_init(0.05)
    prm.max_K = 4096
    with pytest.raises(P.KsError) as e:
        P.ks_scan_batch(ctx.handle, x, d, 1, prm, out)
    assert e.value.code == P.KS_E_RANGE
    prm = P.ks_params_init(0.05)
    prm.alpha = 1.5
    with pytest.raises(P.KsError) as e:
        P.ks_scan_batch(ctx.handle, x, d, 1, prm, out)
    assert e.value.code == P.KS_E_INVALID
    with pytest.raises(ValueError):
        P.ks_scan_batch(ctx.handle, x, d, 2, P.ks_params_init(0.05), out)  # out too small
    with pytest.raises(P.KsError) as e:
        P.ks_launch_set(ctx.handle, 64, 1, P.KS_LAUNCH_GRID, 1 << 20, 0, variant=P.KS_SCAN_VARIANTS)
    assert e.value.code == P.KS_E_RANGE


def test_deterministic(ctx):
    b = S.make_batch(3, num_series=64, first_series=500)
    x, d = batch_arrays(b)
    runs = [run_gpu(ctx, x, d, max_K=512, launch=ln) for ln in LAUNCHES + [LAUNCHES[4]]]
    for g, u in runs[1:]:
        assert g.tobytes() == runs[0][0].tobytes() and np.array_equal(u, runs[0][1])


def test_device_generator_matches_host(dev):
    import torch

    for recipe, num in [(1, 1), (3, 20), (5, 2)]:
        b = S.make_batch(recipe, num_series=num)
        x = S.fill_host(b)
        buf = torch.empty(b.total_elems, dtype=torch.int32, device="cuda")
        S.fill_device(b, buf.data_ptr(), b.total_elems)
        y = buf.cpu().numpy().view(np.uint32)
        for t in range(num):
            assert np.array_equal(S.series_view(x, b, t), S.series_view(y, b, t)), (recipe, t)

"""GPU parity of the proposal network (forward, backward, training step) through the C ABI.

Two bars, neither a hand-picked tolerance:

* Bit-exact on grid cases. Weights, biases, features and logit gradients are
  small multiples of powers of two, chosen so that every FP32 sum the device
  makes is exact in any order (oracle.cnn.exact_in_fp32 checks this on the
  oracle side first). The device logits and gradients must then equal the
  oracle's bit for bit: a wrong tap, edge row, channel or layer shows.
* Layer by layer on realistic inputs (decile features of generated series,
  trained and freshly initialised networks), through ks_cnn_trace: each
  layer's output is checked against the exact value computed here from the
  device's OWN inputs to that layer. An FP32 sum of n exact products lies
  within gamma(n) sum |terms| of the exact sum in any order (oracle.cnn: one
  ulp per addition), so an fp32 output must lie within that radius and a
  stored bf16 activation between the roundings of the radius' ends (at most
  one bf16 step, and only where a rounding boundary falls inside). A wrong
  tap, mask or row moves values by far more.
"""

from pathlib import Path

import numpy as np
import pytest

import oracle as O
import paper_2511_05958_amd as P
from oracle import cnn as C
from paper_2511_05958_amd import synth as S

pytestmark = pytest.mark.gpu

MODELS = Path(__file__).resolve().parent.parent / "paper_2511_05958_amd" / "models"
NA, NG = P.KS_CNN_TRACE_ACTS, P.KS_CNN_TRACE_GRADS
DW_GRID = 256  # workgroups (partial sums) of a device weight-gradient sum


@pytest.fixture(scope="module")
def ctx(dev):
    c = P.Context(0)
    yield c
    c.close()


def slot_rows(max_K):
    return (max_K + 4 + 15) // 16 * 16


def dw_chain(rows):
    """Additions on the longest path of a device weight-gradient sum over `rows`
    slot rows: workgroup g adds the rows of its 64-row tiles in 32-row
    matrix-core steps (tiles g, g + G, ...), then the G partial sums are added,
    so every term passes through at most ceil(tiles / G) 64 + G additions (an
    FP32 summation tree of that depth stays within gamma(depth) sum |terms|)."""
    tiles = -(-rows // 64)
    G = min(tiles, DW_GRID)
    return -(-tiles // G) * 64 + G + 1


def grid_case(seed, Ks, dl_frac=0.05):
    """Grid-valued parameters (weights in s {-1, 0, 1}, position-channel weights
    0, biases on the products' grid), integer features 0..7 and sparse logit
    gradients in 2^-4 {-3..3}."""
    rng = np.random.default_rng(seed)
    scales, dens = (2.0 ** -2, 2.0 ** -3, 2.0 ** -3, 2.0 ** -3), (0.6, 0.3, 0.3, 0.5)
    parts = []
    for l, (cin, cout) in enumerate(C.LAYERS):
        W = rng.choice([-1.0, 0.0, 1.0], size=(cout, cin, C.KW), p=[dens[l] / 2, 1 - dens[l], dens[l] / 2]) * scales[l]
        if l == 0:
            W[:, 9:, :] = 0.0
        b = rng.integers(-4, 5, cout) * scales[l] * (1.0 if l == 0 else 0.25)
        parts += [W, b.astype(np.float64)]
    theta = C.pack(parts)
    feats = [rng.integers(0, 8, (K, 9)).astype(np.float32) for K in Ks]
    dzs = [np.where(rng.random(K) < dl_frac, rng.integers(-3, 4, K) * 2.0 ** -4, 0.0) for K in Ks]
    return theta, feats, dzs


def desc_for(Ks):
    return P.make_desc(np.zeros(len(Ks), np.int64), Ks, np.ones(len(Ks), np.int64))


def fdev(a):
    import torch

    return P.to_device(np.ascontiguousarray(a, np.float32).ravel()).view(torch.float32)


def device_logits(ctx, theta, feats, max_K):
    import torch

    Ks = [len(f) for f in feats]
    d = desc_for(Ks)
    lg = torch.full((sum(Ks),), float("nan"), dtype=torch.float32, device="cuda")
    with P.Model(ctx, seed=0) as m:
        P.ks_model_set_params(m.handle, theta.astype(np.float32))
        P.ks_cnn_forward(ctx.handle, m.handle, fdev(np.concatenate(feats)), P.to_device(d), len(Ks), max_K, lg)
        torch.cuda.synchronize()
    z = lg.cpu().numpy().astype(np.float64)
    return [z[int(a):int(a) + K] for a, K in zip(d["aux_offset"], Ks)]


def device_grads(ctx, theta, feats, dzs, max_K):
    import torch

    Ks = [len(f) for f in feats]
    d = desc_for(Ks)
    g = torch.full((P.KS_CNN_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
    with P.Model(ctx, seed=0) as m:
        P.ks_model_set_params(m.handle, theta.astype(np.float32))
        P.ks_cnn_backward(ctx.handle, m.handle, fdev(np.concatenate(feats)), P.to_device(d), len(Ks), max_K,
                          fdev(np.concatenate(dzs)), g)
        torch.cuda.synchronize()
    return g.cpu().numpy().astype(np.float64)


def device_trace(ctx, theta, feats, max_K, dzs=None, labels=None):
    """Per series: acts [K][NA], grads_in [K][NG] (None without a backward), and the parameter gradient."""
    import torch

    Ks = [len(f) for f in feats]
    rows = sum(Ks)
    d = desc_for(Ks)
    acts = torch.full((rows * NA,), float("nan"), dtype=torch.float32, device="cuda")
    bwd = dzs is not None or labels is not None
    gin = torch.full((rows * NG,), float("nan"), dtype=torch.float32, device="cuda") if bwd else None
    g = torch.full((P.KS_CNN_PARAMS,), float("nan"), dtype=torch.float32, device="cuda") if bwd else None
    with P.Model(ctx, seed=0) as m:
        P.ks_model_set_params(m.handle, theta.astype(np.float32))
        P.ks_cnn_trace(ctx.handle, m.handle, fdev(np.concatenate(feats)), P.to_device(d), len(Ks), max_K,
                       labels=None if labels is None else torch.tensor(labels, dtype=torch.int32, device="cuda"),
                       dlogits=None if dzs is None else fdev(np.concatenate(dzs)), acts=acts, grads_in=gin, grads=g)
        torch.cuda.synchronize()
    a = acts.cpu().numpy().astype(np.float64).reshape(rows, NA)
    gi = gin.cpu().numpy().astype(np.float64).reshape(rows, NG) if bwd else None
    out = []
    for off, K in zip(d["aux_offset"], Ks):
        off = int(off)
        out.append((a[off:off + K], None if gi is None else gi[off:off + K]))
    return out, (g.cpu().numpy().astype(np.float64) if bwd else None)


# ------------------------------------------------------------------ grid cases: bit-exact


@pytest.mark.parametrize("max_K,Ks", [(64, [2, 3, 5, 17, 64]), (256, [1, 40, 129, 256, 7]),
                                      (512, [300, 509, 66]), (1024, [1000, 1024, 3]), (2048, [2048, 1500])],
                         ids=["maxK64", "maxK256", "maxK512", "maxK1024", "maxK2048"])
def test_forward_grid_bit_exact(ctx, max_K, Ks):
    """ks_cnn_forward (the fused inference kernel: tiles of 128 rows that span
    series slots) and the per-layer training forward (ks_cnn_trace) on grid
    cases at every K class: logits bit-exact with the oracle. A K = 1 series is
    skipped (no candidate split): its logit row is not written."""
    theta, feats, _ = grid_case(7 + max_K, Ks)
    caches = [C.forward(f, theta, round_bf16=True) for f in feats]
    assert C.exact_in_fp32([c for (_, c), K in zip(caches, Ks) if K >= 2], theta)
    z = device_logits(ctx, theta, feats, max_K)
    tr, _ = device_trace(ctx, theta, feats, max_K)
    nontrivial = 0
    for K, zg, (zo, _), (a, _) in zip(Ks, z, caches, tr):
        if K < 2:
            assert np.all(np.isnan(zg)) and np.all(np.isnan(a))  # skipped: rows left as they were
            continue
        assert np.array_equal(zg, zo), (K, np.max(np.abs(zg - zo)))
        assert np.array_equal(a[:, NA - 1], zo), K
        nontrivial += int(np.ptp(zo) > 0)
    assert nontrivial >= 2
    # every layer has ReLU units on both sides of zero (the masks matter)
    for l in range(3):
        y = np.concatenate([c["y"][l].ravel() for _, c in caches])
        assert 0.2 < np.mean(y > 0) < 0.8


@pytest.mark.parametrize("Ks,dl", [([5, 17, 65, 129], 0.05), ([3, 5, 9, 17, 33, 65], 0.2)], ids=["tiles", "edges"])
@pytest.mark.parametrize("seed", [0, 1])
def test_backward_grid_bit_exact(ctx, Ks, dl, seed):
    """ks_cnn_backward on grid cases: every weight and bias gradient of every
    layer bit-exact (input-gradient convolutions with flipped taps, ReLU masks,
    weight-gradient sums over every row of the batch and their partials)."""
    theta, feats, dzs = grid_case(100 + seed, Ks, dl)
    caches = [C.forward(f, theta, round_bf16=True) for f in feats]
    assert C.exact_in_fp32([c for _, c in caches], theta, dzs)
    go = np.zeros(C.NUM_PARAMS)
    for (_, cache), dz in zip(caches, dzs):
        go += C.backward(dz, theta, cache, round_bf16=True)
    g = device_grads(ctx, theta, feats, dzs, 256)
    bad = np.nonzero(g != go)[0]
    assert bad.size == 0, (bad[:10], g[bad[:5]], go[bad[:5]])
    for part in C.unpack(go)[0::2]:  # every layer's weights receive a non-zero gradient
        assert np.count_nonzero(part) > 0


# ------------------------------------------------------------------ realistic inputs: layer by layer


def realistic_case(kind, seed):
    if kind == "recipe2":
        b = S.make_batch(2, num_series=4, first_series=60 + seed)
        max_K, model = 256, "proposal_r4.ckpt"
    elif kind == "recipe3":
        b = S.make_batch(3, num_series=12, first_series=70 + seed)
        max_K, model = 512, "proposal_r3.ckpt"
    else:
        b = S.make_batch(5, num_series=2, first_series=80 + seed)
        max_K, model = 1024, "proposal_r5.ckpt"
    x = S.fill_host(b)
    feats = []
    for t in range(b.num_series):
        o, K, N = int(b.specs["offset"][t]), int(b.specs["K"][t]), int(b.specs["N"][t])
        feats.append(O.features(x[o:o + K * N].reshape(K, N)))
    return feats, max_K, model


def load_theta(ctx, name, seed=0):
    with P.Model(ctx, seed=seed) as m:
        if name != "init":
            P.ks_model_load(m.handle, MODELS / name)
        return P.ks_model_get_params(m.handle).astype(np.float64)


def split_acts(a):
    """acts rows [K][NA] -> x0 [11][K], a1, a2, a3 [64][K], z [K]."""
    return a[:, :11].T, a[:, 11:75].T, a[:, 75:139].T, a[:, 139:203].T, a[:, 203]


def check_forward_layers(f, theta, a):
    """Every layer of one series' device forward against the exact value on its own inputs."""
    x0, a1, a2, a3, z = split_acts(a)
    assert np.array_equal(x0, C.bf16(C.network_input(f)))  # features and position channels
    moved = 0
    for l, (xin, aout) in enumerate([(x0, a1), (a1, a2), (a2, a3)]):
        y, r = C.layer_forward(xin, theta, l)
        lo, hi = C.activation_interval(y, r)
        assert np.all((aout >= lo) & (aout <= hi)), (l, int(np.sum((aout < lo) | (aout > hi))))
        moved += int(np.sum(aout != C.bf16(np.maximum(y, 0.0))))
    y, r = C.layer_forward(a3, theta, 3)
    assert np.all(np.abs(z - y[0]) <= r[0]), float(np.max(np.abs(z - y[0]) / np.maximum(r[0], 1e-300)))
    return moved


def check_backward_layers(theta, a, gi, dz):
    """Every layer of one series' device backward on its own inputs. Returns the
    per-layer (output gradient, input) pairs for the weight-gradient check."""
    x0, a1, a2, a3, _ = split_acts(a)
    K = a.shape[0]
    assert np.array_equal(gi[:, 0], dz)
    dys = [gi[:, 1:65].T, gi[:, 65:129].T, gi[:, 129:193].T]  # at y2, y1, y0
    src = [dz[None, :], dys[0], dys[1]]  # output gradients of layers 3, 2, 1
    masks = [a3 != 0, a2 != 0, a1 != 0]
    for j, l in enumerate((3, 2, 1)):
        dx, r = C.input_grad(src[j], theta, l, K)
        m = masks[j]
        assert np.all(dys[j][~m] == 0.0), l
        err = np.abs(dys[j] - dx)[m]
        assert np.all(err <= r[m]), (l, float(np.max(err / np.maximum(r[m], 1e-300))))
    return [(src[0], a3), (dys[0], a2), (dys[1], a1), (dys[2], x0)]  # layers 3, 2, 1, 0


def check_weight_grads(g, pairs_per_series, n_add):
    gp = C.unpack(g)
    for j, l in enumerate((3, 2, 1, 0)):
        dW, rW, db, rb = C.weight_grad([p[j][0] for p in pairs_per_series], [p[j][1] for p in pairs_per_series], n_add)
        assert np.all(np.abs(gp[2 * l] - dW) <= rW), (l, float(np.max(np.abs(gp[2 * l] - dW) / np.maximum(rW, 1e-300))))
        assert np.all(np.abs(gp[2 * l + 1] - db) <= rb), l
        assert np.median(rW) < 1e-3 * np.max(np.abs(dW))  # not vacuous


@pytest.mark.parametrize("kind", ["recipe2", "recipe3", "recipe5"])
@pytest.mark.parametrize("weights", ["trained", "init"])
def test_forward_layers_on_device_inputs(ctx, kind, weights):
    """Per-layer forward (training kernels) checked layer by layer; the fused
    inference kernel's logits equal the per-layer kernels' bit for bit (same
    operands, same order of matrix-core steps, bias added last)."""
    feats, max_K, model = realistic_case(kind, 0)
    theta = load_theta(ctx, model if weights == "trained" else "init", 31)
    tr, _ = device_trace(ctx, theta, feats, max_K)
    z = device_logits(ctx, theta, feats, max_K)
    moved, total = 0, 0
    for f, (a, _), zf in zip(feats, tr, z):
        moved += check_forward_layers(f, theta, a)
        total += 3 * 64 * len(f)
        assert np.array_equal(zf, a[:, NA - 1])
    assert moved <= 0.05 * total, (moved, total)  # most activations are the rounding of the exact value


@pytest.mark.parametrize("kind", ["recipe2", "recipe3"])
def test_backward_layers_on_device_inputs(ctx, kind):
    feats, max_K, model = realistic_case(kind, 2)
    theta = load_theta(ctx, model)
    rng = np.random.default_rng(5)
    dzs = [rng.normal(0, 1e-2, len(f)).astype(np.float32).astype(np.float64) for f in feats]
    tr, g = device_trace(ctx, theta, feats, max_K, dzs=dzs)
    pairs = []
    for f, (a, gi), dz in zip(feats, tr, dzs):
        check_forward_layers(f, theta, a)
        pairs.append(check_backward_layers(theta, a, gi, dz))
    check_weight_grads(g, pairs, dw_chain(len(feats) * slot_rows(max_K)))
    # ks_cnn_backward runs the same kernels: the same gradient bit for bit
    assert np.array_equal(device_grads(ctx, theta, feats, dzs, max_K), g)


def test_train_step_on_device_inputs(ctx):
    """ks_train_step: its gradient equals the trace's (same kernels), whose
    softmax logit gradient lies within the FP32 bound of the exact gradient of
    the device's own logits and whose layers pass the per-layer checks; the
    loss likewise; then one Adam update on the device's own gradient."""
    import torch

    b = S.make_batch(2, num_series=8, first_series=200)
    x = S.fill_host(b)
    feats, labels = [], []
    for t in range(b.num_series):
        o, K, N = int(b.specs["offset"][t]), int(b.specs["K"][t]), int(b.specs["N"][t])
        r = x[o:o + K * N].reshape(K, N)
        feats.append(O.features(r))
        res = O.scan_series(r)
        labels.append(int(res["cp"]) if res["significant"] else -1)
    nsig = sum(c >= 1 for c in labels)
    assert 3 <= nsig < len(labels)
    theta = load_theta(ctx, "proposal_r4.ckpt")
    tr, gt = device_trace(ctx, theta, feats, 256, labels=labels)
    d = P.make_desc(b.specs["offset"], b.specs["K"], b.specs["N"])
    with P.Model(ctx, seed=0) as m:
        P.ks_model_set_params(m.handle, theta.astype(np.float32))  # fresh Adam state
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        lr = 1e-3
        P.ks_train_step(ctx.handle, m.handle, fdev(np.concatenate(feats)), P.to_device(d),
                        torch.tensor(labels, dtype=torch.int32, device="cuda"), b.num_series, 256, lr, loss)
        torch.cuda.synchronize()
        g = P.ks_model_grads(m.handle).astype(np.float64)
        theta1 = P.ks_model_get_params(m.handle).astype(np.float64)
    assert np.array_equal(g, gt)
    pairs, lc, rl, labs = [], 0.0, 0.0, 0.0
    for f, (a, gi), c in zip(feats, tr, labels):
        check_forward_layers(f, theta, a)
        if c < 1:
            assert np.all(gi == 0.0)  # not significant: no gradient
            pairs.append(check_backward_layers(theta, a, gi, np.zeros(len(f))))
            continue
        dz, rdz, ls, rls = C.softmax_grad(a[:, NA - 1], c, nsig)
        assert np.all(np.abs(gi[:, 0] - dz) <= rdz), float(np.max(np.abs(gi[:, 0] - dz) / np.maximum(rdz, 1e-300)))
        pairs.append(check_backward_layers(theta, a, gi, gi[:, 0]))
        lc, rl, labs = lc + ls, rl + rls, labs + abs(ls)
    rl += C.gamma(nsig) * labs  # the per-series terms are added up in FP32
    assert abs(float(loss.cpu()[0]) - lc) <= rl, (float(loss.cpu()[0]), lc, rl)
    check_weight_grads(g, pairs, dw_chain(b.num_series * slot_rows(256)))
    # Adam from zero moments on the device's own gradient: the FP32 update
    # lr (m / bc1) / (sqrt(v / bc2) + eps) passes through at most 16 roundings
    # and constants (0.1f, 0.001f, 1e-8f) each within one ulp, so it lies within
    # 16 2^-24 of the exact update; the new parameter adds half an ulp of itself
    th, _, _ = C.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), g, 1, lr)
    bound = 16 * 2.0 ** -24 * np.abs(th - theta) + 2.0 ** -24 * (np.abs(th) + np.abs(theta1))
    assert np.all(np.abs(theta1 - th) <= bound)

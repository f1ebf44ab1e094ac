"""Pins of the proposal-network oracle (oracle/cnn.py) and the feature oracle.

Independent references: numpy sort for the deciles; torch's bfloat16
conversion, torch.nn.functional.conv1d and torch.autograd in float64 on the
CPU for the network; central finite differences; torch.optim.Adam.
"""

import numpy as np
import pytest
import torch

import oracle as O
from oracle import cnn as C


def rand_theta(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, C.NUM_PARAMS)


def torch_net(theta, feat, round_bf16):
    P = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in C.unpack(theta)]
    a = torch.tensor(C.network_input(feat)[None], dtype=torch.float64)

    def rnd(t):
        return t.float().bfloat16().double() if round_bf16 else t

    for l in range(4):
        W = P[2 * l]
        y = torch.nn.functional.conv1d(rnd(a), rnd(W) if round_bf16 else W, P[2 * l + 1], padding=C.PAD)
        a = torch.relu(y) if l < 3 else y
    return a[0, 0], P


def test_features_match_numpy_deciles():
    rng = np.random.default_rng(0)
    for K, N in [(3, 1), (4, 7), (17, 64), (5, 1000)]:
        r = rng.integers(50, 5000, (K, N), dtype=np.uint32)
        f = O.features(r)
        m = int(r.min())
        s = np.sort(r, axis=1).astype(np.int64)
        idx = [(k * (N - 1)) // 10 for k in range(1, 10)]
        ref = ((s[:, idx] - m) / max(m, 1)).astype(np.float32)
        assert np.array_equal(f, ref)
        assert (np.diff(f, axis=1) >= 0).all() and (f >= 0).all()


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 3, 5000), rng.normal(0, 1e-3, 1000), [0.0, -0.0, 1.0, 65504.0]])
    # exact ties of the 16-bit truncation, both parities
    t = np.array([0x3F808000, 0x3F818000, 0xBF808000, 0x40008000], np.uint32).view(np.float32)
    x = np.concatenate([x, t.astype(np.float64)])
    ref = torch.tensor(x, dtype=torch.float64).float().bfloat16().double().numpy()
    assert np.array_equal(C.bf16(x), ref)


@pytest.mark.parametrize("round_bf16", [False, True])
def test_forward_matches_torch_conv1d(round_bf16):
    rng = np.random.default_rng(2)
    theta = rand_theta(3)
    feat = rng.random((37, 9)).astype(np.float32)
    z, _ = C.forward(feat, theta, round_bf16)
    zt, _ = torch_net(theta, feat, round_bf16)
    # intermediate FP32 rounding of activations exists only in the oracle's bf16 mode
    tol = 1e-12 if not round_bf16 else 5e-2 * np.abs(z).max()
    assert np.max(np.abs(z - zt.detach().numpy())) <= tol


def test_backward_matches_autograd_and_finite_differences():
    rng = np.random.default_rng(4)
    theta = rand_theta(5)
    feats = [rng.random((K, 9)).astype(np.float32) for K in (12, 20)]
    labels = [5, 13]
    loss, g = C.batch_loss_grad(feats, labels, theta, round_bf16=False)
    # torch autograd on the same FP64 network
    tot = 0.0
    Ps = None
    gt = np.zeros(C.NUM_PARAMS)
    for feat, c in zip(feats, labels):
        z, P = torch_net(theta, feat, False)
        lz = torch.log_softmax(z[1:], 0)
        l = -lz[c - 1] / len(labels)
        l.backward()
        gt += np.concatenate([p.grad.numpy().ravel() for p in P])
        tot += float(l.detach())
    assert abs(loss - tot) < 1e-12
    assert np.max(np.abs(g - gt)) <= 1e-10 * np.max(np.abs(gt))
    # central differences on a sample of coordinates
    for j in rng.choice(C.NUM_PARAMS, 40, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[j] += h
        tm[j] -= h
        fd = (C.batch_loss_grad(feats, labels, tp, False)[0] - C.batch_loss_grad(feats, labels, tm, False)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-8, j


def he_theta(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in C.LAYERS:
        parts.append(rng.normal(0, np.sqrt(2.0 / (cin * C.KW)), (cout, cin, C.KW)))
        parts.append(np.zeros(cout))
    return C.pack(parts)


def test_bf16_backward_close_to_exact():
    # sanity check of the rounding placement: bf16 operands perturb, not redirect, the gradient
    rng = np.random.default_rng(6)
    theta = he_theta(7)
    feats = [rng.random((30, 9)).astype(np.float32)]
    _, g0 = C.batch_loss_grad(feats, [9], theta, round_bf16=False)
    _, g1 = C.batch_loss_grad(feats, [9], theta, round_bf16=True)
    cos = g0 @ g1 / (np.linalg.norm(g0) * np.linalg.norm(g1))
    assert cos > 0.99


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    theta = rng.normal(size=50)
    g1, g2 = rng.normal(size=50), rng.normal(size=50)
    p = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    th = theta.copy()
    for step, g in enumerate([g1, g2], start=1):
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = C.adam_step(th, m, v, g, step, 1e-3)
    assert np.max(np.abs(th - p.detach().numpy())) < 1e-14


def test_position_channels():
    x = C.network_input(np.zeros((5, 9), np.float32))
    assert x.shape == (11, 5)
    assert np.allclose(x[9], [0, 0.25, 0.5, 0.75, 1.0]) and np.allclose(x[10], [0, 0.64, 0.96, 0.96, 0.64])


def test_propose_mass():
    z = np.array([100.0, 0.0, 1.0, 5.0, 1.0, 0.0, -3.0])
    c, conf = C.propose(z, 1)
    p = np.exp(z[1:] - z[1:].max())
    p /= p.sum()
    assert c == 3 and abs(conf - p[1:4].sum()) < 1e-15


def test_refine_window_and_fallback():
    rng = np.random.default_rng(9)
    r = rng.integers(100, 130, (64, 16), dtype=np.uint32)
    r[40:] += 40
    res, U = O.scan_series(r, want_allU=True)
    full = O.refine(U, 64, 20, 0.1, 8, 0.5)          # low confidence: full scan
    assert not full["refined"] and (full["cp"], full["U"]) == (res["cp"], res["U"])
    hit = O.refine(U, 64, 38, 0.9, 8, 0.5)           # window [30, 46] holds c* = 40
    assert hit["refined"] and (hit["cp"], hit["U"], hit["p"]) == (res["cp"], res["U"], res["p"])
    miss = O.refine(U, 64, 10, 0.9, 3, 0.5)          # window [7, 13] misses c*
    lam = [U[c] ** 2 / (c * (64 - c)) for c in range(7, 14)]
    assert miss["refined"] and miss["cp"] == 7 + int(np.argmax(lam))
    assert not O.refine(U, 64, 10, float("nan"), 3, 0.5)["refined"]  # NaN confidence falls back
    edge = O.refine(U, 64, 1, 1.0, 8, 0.0)           # window clipped to [1, 9]
    assert 1 <= edge["cp"] <= 9


# ---------------------------------------------------------------- error-bound pins
#
# The per-layer radii of oracle.cnn are checked against an FP32 emulation that
# sums the same terms in random orders, with round-to-nearest and with
# truncation toward zero (the two adders the bound claims to cover). A radius
# missing a term, or counting too few additions, is exceeded by some order.


def _fp32_sums(terms, rng, mode):
    """Sequential float32 sums over axis 0 of `terms` (exact float64 products),
    each output element in its own random order; mode 'rn' or 'rz'."""
    n = terms.shape[0]
    order = np.argsort(rng.random(terms.shape), axis=0)
    t = np.take_along_axis(terms, order, axis=0).astype(np.float32)
    acc = np.zeros(terms.shape[1:], np.float32)
    for k in range(n):
        s = acc.astype(np.float64) + t[k].astype(np.float64)
        r = s.astype(np.float32)
        if mode == "rz":
            over = np.abs(r.astype(np.float64)) > np.abs(s)
            r = np.where(over, np.nextafter(r, np.float32(0)), r)
        acc = r
    return acc.astype(np.float64)


def _conv_terms(x, W, b):
    """All products W[o][i][k] x[i][t + k - 2] and the bias, stacked on axis 0: [cin 5 + 1][cout][K]."""
    cin, K = x.shape
    xp = np.zeros((cin, K + 2 * C.PAD))
    xp[:, C.PAD:C.PAD + K] = x
    terms = [W[:, i, k][:, None] * xp[i, k:k + K][None, :] for i in range(cin) for k in range(C.KW)]
    terms.append(np.repeat(np.asarray(b, np.float64)[:, None], K, axis=1))
    return np.stack(terms)


@pytest.mark.parametrize("mode", ["rn", "rz"])
def test_layer_forward_radius_covers_fp32_orders(mode):
    rng = np.random.default_rng(11)
    theta = he_theta(12)
    x = C.bf16(np.maximum(rng.normal(0, 1, (64, 40)), 0.0))
    for l in (1, 3):
        P_ = C.unpack(theta)
        W, b = C.bf16(P_[2 * l]), P_[2 * l + 1]
        y, r = C.layer_forward(x, theta, l)
        terms = _conv_terms(x, W, b)
        assert np.allclose(terms.sum(axis=0), y, rtol=1e-13, atol=1e-13)
        worst = 0.0
        for _ in range(3):
            e = np.abs(_fp32_sums(terms, rng, mode) - y)
            assert np.all(e <= r)
            worst = max(worst, float(np.max(e / r)))
        assert worst > 1e-4  # random orders reach within four orders of magnitude of the radius
    # a radius that forgets the bias term is exceeded: rebuild without it
    y, r = C.layer_forward(x, theta, 1)
    P_ = C.unpack(theta)
    wrong = (C.gamma(64 * C.KW) + 0) * C.conv(np.abs(x), np.abs(C.bf16(P_[2])), np.zeros(64))
    assert np.all(r >= wrong)


def test_activation_interval_contains_device_roundings():
    rng = np.random.default_rng(13)
    y = rng.normal(0, 4, 20000)
    r = np.abs(y) * 3e-5 + 1e-7
    lo, hi = C.activation_interval(y, r)
    for v in (y - r, y + r, y + r * (2 * rng.random(y.size) - 1)):
        a = C.bf16(np.maximum(C.f32(v), 0.0))
        assert np.all((a >= lo) & (a <= hi))
    # at most one bf16 step wide where the radius is below half a step
    step = np.maximum(np.abs(lo), np.abs(hi)) * 2.0 ** -7
    assert np.all(hi - lo <= step)


@pytest.mark.parametrize("mode", ["rn", "rz"])
def test_input_and_weight_grad_radii_cover_fp32_orders(mode):
    rng = np.random.default_rng(14)
    theta = he_theta(15)
    K = 33
    P_ = C.unpack(theta)
    dyf = C.f32(rng.normal(0, 1e-2, (64, K)))
    dx, r = C.input_grad(dyf, theta, 2, K)
    # terms of dx[i][t] = sum_{o,k} W[o][i][k] dr[o][t - k + 2]
    W, dr = C.bf16(P_[4]), C.bf16(dyf)
    dyp = np.zeros((64, K + 4))
    dyp[:, 2:2 + K] = dr
    terms = np.stack([W[o, :, k][:, None] * dyp[o, 4 - k:4 - k + K][None, :] for o in range(64) for k in range(C.KW)])
    assert np.allclose(terms.sum(axis=0), dx, rtol=1e-13, atol=1e-18)
    for _ in range(2):
        assert np.all(np.abs(_fp32_sums(terms, rng, mode) - dx) <= r)
    # weight gradient over two series: dW[o][i][k] = sum_t dr[o][t] x[i][t + k - 2]
    xs = [C.bf16(np.maximum(rng.normal(0, 1, (64, K)), 0.0)), C.bf16(np.maximum(rng.normal(0, 1, (64, 20)), 0.0))]
    dyfs = [dyf, C.f32(rng.normal(0, 1e-2, (64, 20)))]
    dW, rW, db, rb = C.weight_grad(dyfs, xs, n_add=K + 20 + 8)
    prods = []
    for d_, x_ in zip(dyfs, xs):
        Kx = x_.shape[1]
        xp = np.zeros((64, Kx + 4))
        xp[:, 2:2 + Kx] = x_
        for t in range(Kx):
            prods.append(C.bf16(d_)[:, t][:, None, None] * np.stack([xp[:, t + k] for k in range(C.KW)], axis=1)[None])
    prods = np.stack(prods)  # [rows][o][i][k]
    assert np.allclose(prods.sum(axis=0), dW, rtol=1e-12, atol=1e-20)
    e = np.abs(_fp32_sums(prods[:, :8, :8, :], rng, mode) - dW[:8, :8, :])
    assert np.all(e <= rW[:8, :8, :])
    bsum = np.concatenate([d_ for d_ in dyfs], axis=1).T  # [rows][o]
    assert np.all(np.abs(_fp32_sums(bsum, rng, mode) - db) <= rb)


def test_softmax_grad_covers_float32_evaluation():
    rng = np.random.default_rng(16)
    for K, scale in [(5, 1.0), (64, 3.0), (256, 8.0), (1024, 20.0)]:
        z = rng.normal(0, scale, K)
        lab = int(rng.integers(1, K))
        nsig = int(rng.integers(1, 9))
        d, rd, loss, rl = C.softmax_grad(z, lab, nsig)
        # exact values: the gradient of the mean cross-entropy (the oracle's loss_and_dlogits)
        lo, dlo = C.loss_and_dlogits(z, lab)
        assert abs(loss - lo / nsig) <= 1e-13 * max(1.0, abs(loss))
        assert np.allclose(d, dlo / nsig, rtol=1e-12, atol=1e-300)
        # a float32 evaluation as the device does it, exponentials perturbed by up to one ulp
        zf = z.astype(np.float32)
        for trial in range(4):
            mx = zf[1:].max()
            xx = (zf[1:] - mx).astype(np.float32)
            e = np.exp2((xx * np.float32(1.4426950408889634)).astype(np.float32)).astype(np.float32)
            e = e * (1 + (trial - 1.5) / 1.5 * 2.0 ** -23 * rng.random(e.size)).astype(np.float32)
            s = np.float32(0)
            for v in e[rng.permutation(e.size)]:
                s = np.float32(s + v)
            p = (e / s).astype(np.float32)
            q = (p - (np.arange(1, K) == lab).astype(np.float32)).astype(np.float32)
            dd = (q * np.float32(1.0 / nsig)).astype(np.float32)
            assert np.all(np.abs(dd.astype(np.float64) - d[1:]) <= rd[1:]), (K, trial)
            lf = np.float32((np.float32(np.log(s)) - np.float32(zf[lab] - mx)) * np.float32(1.0 / nsig))
            assert abs(float(lf) - loss) <= rl, (K, trial)


def test_dyadic_quantum_and_exactness_precondition():
    assert C.dyadic_quantum([0.75, 3.0, 0.0]) == 0.25
    assert C.dyadic_quantum([1.5, 2.0 ** -10]) == 2.0 ** -10
    assert C.dyadic_quantum([6.0, 12.0]) == 2.0 and C.dyadic_quantum([0.0]) == np.inf
    rng = np.random.default_rng(17)
    # a grid case: exact in float32 in every order (emulated), so the oracle's values are the float32 ones
    parts = []
    for l, (cin, cout) in enumerate(C.LAYERS):
        W = rng.choice([-1.0, 0.0, 1.0], size=(cout, cin, C.KW)) * (2.0 ** -2 if l == 0 else 2.0 ** -3)
        if l == 0:
            W[:, 9:, :] = 0.0
        parts += [W, rng.integers(-4, 5, cout) * 2.0 ** -4]
    theta = C.pack(parts)
    feat = rng.integers(0, 8, (24, 9)).astype(np.float32)
    z, cache = C.forward(feat, theta, round_bf16=True)
    assert C.exact_in_fp32([cache], theta)
    x = cache["x"][1]
    P_ = C.unpack(theta)
    terms = _conv_terms(x, C.bf16(P_[2]), P_[3])
    for mode in ("rn", "rz"):
        assert np.array_equal(_fp32_sums(terms, rng, mode), cache["y"][1])
    # Gaussian weights spread the products' exponents over more than 24 bits:
    # not exact, and indeed some float32 order of a layer's sums differs
    theta2 = he_theta(19)
    _, cache2 = C.forward(rng.random((24, 9)).astype(np.float32), theta2, round_bf16=True)
    assert not C.exact_in_fp32([cache2], theta2)
    P2 = C.unpack(theta2)
    terms = _conv_terms(cache2["x"][1], C.bf16(P2[2]), P2[3])
    assert not np.array_equal(_fp32_sums(terms, rng, "rz"), cache2["y"][1])


def test_forward_matches_torch_conv1d_exactly_on_grid():
    """On grid values every FP64 sum is exact, so the oracle's bf16 forward and
    torch's conv1d over torch's own bfloat16 conversions agree bit for bit."""
    rng = np.random.default_rng(18)
    parts = []
    for l, (cin, cout) in enumerate(C.LAYERS):
        W = rng.choice([-1.0, 0.0, 1.0], size=(cout, cin, C.KW)) * 2.0 ** -3
        parts += [W, rng.integers(-4, 5, cout) * 2.0 ** -5]
    theta = C.pack(parts)
    feat = rng.integers(0, 8, (37, 9)).astype(np.float32)
    z, _ = C.forward(feat, theta, round_bf16=True)
    zt, _ = torch_net(theta, feat, True)
    assert np.array_equal(z, zt.detach().numpy())
    assert np.ptp(z) > 0


def test_propose_mass_closed_form():
    """Logits ln t give softmax probabilities t / (K (K - 1) / 2) over rows
    1..K-1: the argmax is K - 1 and the mass within w of it is the sum of the
    window's t over that total."""
    for K, w in [(10, 2), (64, 8), (300, 20)]:
        z = np.log(np.maximum(np.arange(K, dtype=np.float64), 1.0))
        z[0] = 50.0  # row 0 is not a candidate
        c, conf = C.propose(z, w)
        assert c == K - 1
        assert abs(conf - sum(range(K - 1 - w, K)) / (K * (K - 1) / 2)) < 1e-13

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

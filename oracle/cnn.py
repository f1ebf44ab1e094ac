"""Oracle of the learned proposal network (TEST INFRASTRUCTURE; see oracle/__init__.py).

The paper has no learned stage: the network shortlists candidate change
points, which the paper mentions as a way to cut the K-S evaluation
(workflow step 4, last paragraph) and omits because its data are small. It is
a 1-D CNN over the per-row decile features plus two position channels
(t / (K-1) and 4 t (K - t) / K^2, computed in double and rounded to float:
the K-S choice favours central splits, lambda^2 = D^2 c (K - c) / K):

    conv(11 -> 64) ReLU, conv(64 -> 64) ReLU, conv(64 -> 64) ReLU, conv(64 -> 1)

every conv with kernel 5, zero padding 2, bias; one logit per row t. The
proposal is the softmax over rows t = 1..K-1 (the candidate change points).

Numerics mirrored here: every matrix-core operand is rounded to bfloat16
(round to nearest even) - the layer inputs, the weights, and in the backward
pass the output gradients - while sums are exact here (FP64) and FP32 on the
device. Activations between layers are FP32 before that rounding. With
``round_bf16=False`` every rounding is skipped (the plain FP64 network used by
the finite-difference pins).

Parameter vector layout (float32, 44993 values): W0[64][11][5], b0[64],
W1[64][64][5], b1[64], W2[64][64][5], b2[64], W3[1][64][5], b3[1].
"""

from __future__ import annotations

import numpy as np

KW = 5
PAD = 2
LAYERS = [(11, 64), (64, 64), (64, 64), (64, 1)]


def param_shapes():
    out = []
    for cin, cout in LAYERS:
        out.append((cout, cin, KW))
        out.append((cout,))
    return out


NUM_PARAMS = int(sum(np.prod(s) for s in param_shapes()))
assert NUM_PARAMS == 44993


def network_input(feat):
    """[11][K]: the nine feature columns, then t / (K-1) and 4 t (K - t) / K^2 (float)."""
    feat = np.asarray(feat, np.float64)
    K = feat.shape[0]
    t = np.arange(K, dtype=np.float64)
    p1 = (t / max(K - 1, 1)).astype(np.float32).astype(np.float64)
    p2 = (4.0 * t * (K - t) / (float(K) * float(K))).astype(np.float32).astype(np.float64)
    return np.vstack([feat.T, p1[None], p2[None]])


def unpack(theta):
    theta = np.asarray(theta, np.float64)
    parts, o = [], 0
    for s in param_shapes():
        n = int(np.prod(s))
        parts.append(theta[o:o + n].reshape(s))
        o += n
    return parts


def pack(parts):
    return np.concatenate([np.asarray(p, np.float64).ravel() for p in parts])


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32; returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def conv(x, W, b):
    """y[o][t] = b[o] + sum_{i,k} W[o][i][k] x[i][t + k - PAD] (zero outside 0..K-1)."""
    cin, K = x.shape
    xp = np.zeros((cin, K + 2 * PAD))
    xp[:, PAD:PAD + K] = x
    y = np.tile(np.asarray(b, np.float64)[:, None], (1, K))
    for k in range(KW):
        y += W[:, :, k] @ xp[:, k:k + K]
    return y


def conv_back_data(dy, W, K):
    """dx[i][t] = sum_{o,k} W[o][i][k] dy[o][t - k + PAD] (adjoint of conv in x)."""
    cout = dy.shape[0]
    dyp = np.zeros((cout, K + 2 * PAD))
    dyp[:, PAD:PAD + K] = dy
    cin = W.shape[1]
    dx = np.zeros((cin, K))
    for k in range(KW):
        # x[i][s] feeds y[o][s - k + PAD]
        dx += W[:, :, k].T @ dyp[:, 2 * PAD - k:2 * PAD - k + K]
    return dx


def conv_back_weight(dy, x):
    """dW[o][i][k] = sum_t dy[o][t] x[i][t + k - PAD]; db[o] = sum_t dy[o][t]."""
    cin, K = x.shape
    xp = np.zeros((cin, K + 2 * PAD))
    xp[:, PAD:PAD + K] = x
    dW = np.zeros((dy.shape[0], cin, KW))
    for k in range(KW):
        dW[:, :, k] = dy @ xp[:, k:k + K].T
    return dW, dy.sum(axis=1)


def forward(feat, theta, round_bf16=True):
    """feat [K][9] -> (logits [K], cache). Logits are exact sums of rounded operands."""
    P = unpack(theta)
    rnd = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    a = network_input(feat)  # [11][K]
    cache = {"x": [], "y": []}
    for l in range(4):
        x = rnd(a)
        W = rnd(P[2 * l])
        y = conv(x, W, P[2 * l + 1])
        cache["x"].append(x)
        cache["y"].append(y)
        if l < 3:
            a = np.maximum(y, 0.0)
            if round_bf16:
                a = f32(a)
    return cache["y"][3][0], cache


def loss_and_dlogits(logits, label):
    """Softmax cross-entropy over rows 1..K-1 against the change point `label`."""
    z = np.asarray(logits, np.float64)
    K = len(z)
    zz = z[1:] - z[1:].max()
    p = np.exp(zz) / np.exp(zz).sum()
    loss = -np.log(p[label - 1])
    d = np.zeros(K)
    d[1:] = p
    d[label] -= 1.0
    return loss, d


def backward(dlogits, theta, cache, round_bf16=True):
    """Gradient of sum(dlogits * logits) wrt theta (packed like theta)."""
    P = unpack(theta)
    rnd = bf16 if round_bf16 else (lambda v: np.asarray(v, np.float64))
    K = len(dlogits)
    grads = [None] * 8
    dy = np.asarray(dlogits, np.float64)[None, :]
    for l in range(3, -1, -1):
        dyr = rnd(f32(dy)) if round_bf16 else dy
        dW, db = conv_back_weight(dyr, cache["x"][l])
        grads[2 * l], grads[2 * l + 1] = dW, (f32(dy) if round_bf16 else dy).sum(axis=1)
        if l > 0:
            dx = conv_back_data(dyr, rnd(P[2 * l]), K)
            dy = dx * (cache["y"][l - 1] > 0)
    return pack(grads)


def batch_loss_grad(feats, labels, theta, round_bf16=True):
    """Mean loss and gradient over the series with label >= 1 (label -1: not significant, skipped)."""
    g = np.zeros(NUM_PARAMS)
    total, n = 0.0, sum(1 for c in labels if c >= 1)
    for feat, c in zip(feats, labels):
        if c < 1:
            continue
        z, cache = forward(feat, theta, round_bf16)
        loss, d = loss_and_dlogits(z, c)
        total += loss
        g += backward(d / n, theta, cache, round_bf16)
    return (total / max(n, 1)), g


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, Algorithm 1) with bias correction; step counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def propose(logits, w):
    """(argmax over rows 1..K-1, softmax mass within +-w rows of it)."""
    z = np.asarray(logits, np.float64)
    zz = z[1:] - z[1:].max()
    p = np.exp(zz) / np.exp(zz).sum()
    c = 1 + int(np.argmax(p))
    lo, hi = max(1, c - w), min(len(z) - 1, c + w)
    return c, float(p[lo - 1:hi].sum())

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


# ------------------------------------------------------------------ error bounds
#
# How far may a device evaluation of one layer lie from the exact value? The
# device multiplies the same bf16-rounded operands (layer inputs, weights,
# output gradients) exactly and sums the products in FP32, in an order this
# oracle does not fix (matrix-core steps, then partial sums). Given the
# device's OWN inputs to a layer, the exact sum of its terms is computed here,
# and the device's FP32 sum lies within gamma(n) sum |t_k| of it for ANY order
# of the n additions, each with a relative error of at most u = 2^-23 (one
# FP32 ulp: round-to-nearest and truncating adders alike), with
# gamma(n) = n u / (1 - n u) (Higham, Accuracy and Stability of Numerical
# Algorithms, 2nd ed., Lemma 3.1 and eq. 4.4). Rounding to FP32 and then to
# bf16 (nearest even) is monotone and ReLU is too, so a stored activation lies
# between the roundings of the interval's ends: at most one bf16 step from the
# rounding of the exact value, and equal to it unless a rounding boundary lies
# inside the (narrow) interval. This oracle's own FP64 sums add at most
# n 2^-53 sum |t_k| (counted in the radius too). Matrix cores may read a
# subnormal operand (below 2^-126) as zero and flush subnormal products,
# partial sums and results to zero: the radius also holds every term with a
# subnormal operand and 2^-126 for each of the n + 1 roundings.

U32 = 2.0 ** -23
U64 = 2.0 ** -53
TINY = 2.0 ** -126


def _sub(a):
    """|a| where a is subnormal in float32 (below 2^-126), 0 elsewhere."""
    a = np.abs(np.asarray(a, np.float64))
    return np.where(a < TINY, a, 0.0)


def gamma(n, u=U32):
    nu = float(n) * u
    assert nu < 0.5
    return nu / (1.0 - nu)


def layer_forward(x, theta, l):
    """Pre-activation of layer l on bf16 inputs x [cin][K] (the device's own):
    (y, r) with y the exact sum b + sum W x of the rounded weights and r the
    radius around y within which an FP32 evaluation lies."""
    P = unpack(theta)
    W = bf16(P[2 * l])
    b = np.asarray(P[2 * l + 1], np.float64)
    x = np.asarray(x, np.float64)
    n = W.shape[1] * KW + 1
    s_abs = conv(np.abs(x), np.abs(W), np.abs(b))
    zero = np.zeros_like(b)
    s_sub = conv(_sub(x), np.abs(W), zero) + conv(np.abs(x), _sub(W), _sub(b))
    return conv(x, W, b), (gamma(n) + n * U64) * s_abs + s_sub + (n + 1) * TINY


def activation_interval(y, r):
    """[lo, hi]: the bf16 activations bf16(relu(v)) of every v in [y - r, y + r]."""
    return bf16(np.maximum(y - r, 0.0)), bf16(np.maximum(y + r, 0.0))


def input_grad(dyf, theta, l, K):
    """Gradient at layer l's input from its fp32 output gradient dyf [cout][K]
    (the device's own; the device takes bf16(dyf) as the matrix operand), before
    the ReLU mask of the layer below: (dx, r) as for layer_forward."""
    P = unpack(theta)
    W = bf16(P[2 * l])
    dr = bf16(dyf)
    n = W.shape[0] * KW
    s_abs = conv_back_data(np.abs(dr), np.abs(W), K)
    s_sub = conv_back_data(_sub(dr), np.abs(W), K) + conv_back_data(np.abs(dr), _sub(W), K)
    return conv_back_data(dr, W, K), (gamma(n) + n * U64) * s_abs + s_sub + (n + 1) * TINY


def weight_grad(dyfs, xs, n_add):
    """Weight and bias gradient of one layer over a batch, from each series'
    fp32 output gradient dyf [cout][K] (operand bf16(dyf); the bias gradient
    sums dyf itself) and bf16 input x [cin][K], the device's own. n_add: the
    number of FP32 additions in each device sum (every row the device sums,
    plus its partial sums). Returns (dW, rW, db, rb)."""
    dW = rW = db = rb = 0.0
    sw = sb = 0.0
    rows = 0
    for dyf, x in zip(dyfs, xs):
        dr = bf16(dyf)
        x = np.asarray(x, np.float64)
        w, _ = conv_back_weight(dr, x)
        wa, _ = conv_back_weight(np.abs(dr), np.abs(x))
        ws = conv_back_weight(_sub(dr), np.abs(x))[0] + conv_back_weight(np.abs(dr), _sub(x))[0]
        dW = dW + w
        rW = rW + wa
        sw = sw + ws
        db = db + np.asarray(dyf, np.float64).sum(axis=1)
        rb = rb + np.abs(np.asarray(dyf, np.float64)).sum(axis=1)
        sb = sb + _sub(dyf).sum(axis=1)
        rows += np.asarray(dyf).shape[1]
    c = gamma(n_add) + max(rows, 1) * U64
    return dW, c * rW + sw + (n_add + 1) * TINY, db, c * rb + sb + (n_add + 1) * TINY


def softmax_grad(z, label, nsig):
    """The training step's logit gradient and loss of one series from the
    device's own logits z (rows 0..K-1): softmax over rows 1..K-1,
    d_t = (p_t - [t = label]) / nsig for t >= 1, d_0 = 0, loss
    -log p_label / nsig. Returns (d, rd, loss, rloss): the exact values and the
    radius of an FP32 evaluation that takes m = max z, e_t = exp(z_t - m) by a
    base-2 exponential of the scaled argument (within one ulp), s = sum e_t,
    p_t = e_t / s and (log s - (z_label - m)) / nsig."""
    z = np.asarray(z, np.float64)
    K = len(z)
    x = z[1:] - z[1:].max()
    p = np.exp(x) / np.exp(x).sum()
    # each e_t: the difference, the scaling by log2(e) and the exponential round
    # once each; the sum adds gamma(K - 1); the quotient rounds once
    dx = 2.0 * U32 * (np.abs(x) + 1.0)
    dsum = dx.max() + gamma(K)
    rp = p * (np.exp(dx + dsum) * (1.0 + U32) ** 2 - 1.0)
    onehot = np.zeros(K - 1)
    onehot[label - 1] = 1.0
    q = p - onehot
    inv = 1.0 / nsig
    d = np.zeros(K)
    rd = np.zeros(K)
    d[1:] = q * inv
    # the subtraction and the scaling by the rounded 1 / nsig round once each;
    # exponentials and quotients below the smallest normal float (2^-126) may be
    # flushed to zero or kept subnormal: an absolute 2^-126 per value covers both
    rp = rp + 2.0 ** -126
    rd[1:] = (rp + U32 * (np.abs(q) + rp)) * inv * (1.0 + U32) ** 2 + 2.0 * U32 * np.abs(q) * inv
    s = np.exp(x).sum()
    loss = -np.log(p[label - 1]) * inv
    rloss = (dsum + 2.0 * U32 * (abs(np.log(s)) + abs(x[label - 1]) + 1.0)) * inv + 4.0 * U32 * abs(loss)
    return d, rd, loss, rloss


def dyadic_quantum(a):
    """Largest power of two q with every element of a an integer multiple of q
    (inf for an all-zero array)."""
    a = np.abs(np.asarray(a, np.float64)).ravel()
    a = a[a != 0]
    if a.size == 0:
        return np.inf
    m, e = np.frexp(a)
    v = (m * 2.0 ** 53).astype(np.int64)
    tz = np.zeros(v.shape, np.int64)
    while True:
        odd = (v & 1) == 1
        if odd.all():
            break
        v = np.where(odd, v, v >> 1)
        tz += ~odd
    return 2.0 ** int((e - 53 + tz).min())


def _quanta(a, axis):
    """dyadic_quantum of every slice a[j] along `axis` (inf for all-zero slices)."""
    a = np.moveaxis(np.asarray(a, np.float64), axis, 0)
    return np.array([dyadic_quantum(v) for v in a])


def exact_in_fp32(caches, theta, dzs=None):
    """True when every FP32 sum a device makes for this batch is exact whatever
    its order: the forward pre-activations of each series and, with dzs (the
    logit gradients, one per series), each series' backward input gradients and
    the weight and bias gradient sums over the whole batch. A sum is exact when
    all its terms are multiples of one power of two q and their magnitudes add
    up to less than 2^24 q: then every partial sum is a float32, and the device
    result equals this oracle's bit for bit. q is taken per channel pair (the
    terms of one sum share an output channel; their input channels differ).
    caches: the cache of forward(feat, theta, round_bf16=True) of each series
    (its rounded layer inputs and pre-activations)."""
    P = unpack(theta)
    lim = 2.0 ** 24
    Wr = [bf16(P[2 * l]) for l in range(4)]
    qW = [np.array([[dyadic_quantum(Wr[l][o, i]) for i in range(Wr[l].shape[1])] for o in range(Wr[l].shape[0])])
          for l in range(4)]  # [o][i]
    ok = True
    for cache in caches:
        for l in range(4):
            x, b = cache["x"][l], np.asarray(P[2 * l + 1], np.float64)
            q = np.minimum((qW[l] * _quanta(x, 0)[None, :]).min(axis=1), _quanta(b[:, None], 0))  # per o
            ok &= bool(np.all(conv(np.abs(x), np.abs(Wr[l]), np.abs(b)).max(axis=1) < lim * q))
    if dzs is None:
        return bool(ok)
    # weight-gradient sums run over every row of the batch: magnitudes add up
    sw = [0.0] * 4
    sb = [0.0] * 4
    qd = [np.inf] * 4
    qf = [np.inf] * 4
    qx = [np.inf] * 4
    for cache, dz in zip(caches, dzs):
        K = len(dz)
        d = f32(np.asarray(dz, np.float64)[None, :])
        ok &= bool(np.array_equal(d[0], np.asarray(dz, np.float64)))
        for l in range(3, -1, -1):
            x = cache["x"][l]
            dr = bf16(d)
            w_abs, _ = conv_back_weight(np.abs(dr), np.abs(x))
            sw[l] = sw[l] + w_abs
            sb[l] = sb[l] + np.abs(d).sum(axis=1)
            qd[l] = np.minimum(qd[l], _quanta(dr, 0))
            qf[l] = np.minimum(qf[l], _quanta(d, 0))
            qx[l] = np.minimum(qx[l], _quanta(x, 0))
            if l > 0:
                q = (qW[l] * _quanta(dr, 0)[:, None]).min(axis=0)  # per input channel i
                ok &= bool(np.all(conv_back_data(np.abs(dr), np.abs(Wr[l]), K).max(axis=1) < lim * q))
                d = conv_back_data(dr, Wr[l], K) * (cache["y"][l - 1] > 0)
    for l in range(4):
        ok &= bool(np.all(sw[l].max(axis=2) < lim * qd[l][:, None] * qx[l][None, :]))
        ok &= bool(np.all(sb[l] < lim * qf[l]))
    return bool(ok)

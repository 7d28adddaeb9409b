"""FP64 NumPy oracle of the learned preconditioner's network — TEST
INFRASTRUCTURE ONLY (tests, smoke, bench CPU-baseline leg).

A 4-level 3-D U-Net on a dense box of grid nodes, channels-last tensors
``x[X, Y, Z, C]``:

  level l = 0..3 with channels (16, 32, 64, 128); on the way down two 3x3x3
  convolutions (padding 1) with ReLU, then a 2x2x2 stride-2 convolution with
  ReLU; at the bottom two 3x3x3 convolutions; on the way up a 2x2x2 stride-2
  transposed convolution, channel concatenation [up, skip], two 3x3x3
  convolutions with ReLU; finally a 1x1x1 convolution (no activation).

Convolutions are written from their definition as sums over taps:

  conv:  y[v, o] = b[o] + sum_{t, i} x[s v + t - p, i] W[t, i, o]
  up:    y[2 v + t, o] = b[o] + sum_i x[v, i] W[t, i, o]

with zero padding outside the box; taps t are enumerated with the last
spatial axis fastest.  Backward passes are the exact adjoints, derived by
hand from the same sums (and pinned by finite differences in the tests).
"""
from __future__ import annotations

import numpy as np

CH = (16, 32, 64, 128)
IN_CH = 16   # 5 input channels padded to 16
OUT_CH = 16  # 3 output channels padded to 16


def taps(k):
    r = range(k)
    return [(a, b, c) for a in r for b in r for c in r]


# ---------------------------------------------------------------- layers
def conv(x, W, b, k, s, p):
    """y[v] = b + sum_t x[s v + t - p] @ W[t]; x [X,Y,Z,Ci], W [k^3,Ci,Co]."""
    X, Y, Z, _ = x.shape
    Xo, Yo, Zo = (X + 2 * p - k) // s + 1, (Y + 2 * p - k) // s + 1, (Z + 2 * p - k) // s + 1
    xp = np.pad(x, ((p, p), (p, p), (p, p), (0, 0)))
    y = np.broadcast_to(b, (Xo, Yo, Zo, W.shape[2])).astype(np.float64).copy()
    for ti, (a, bb, c) in enumerate(taps(k)):
        sl = xp[a:a + s * Xo:s, bb:bb + s * Yo:s, c:c + s * Zo:s, :]
        y += sl @ W[ti]
    return y


def conv_backward(x, W, dy, k, s, p):
    """Adjoint of conv: returns (dx, dW, db)."""
    X, Y, Z, _ = x.shape
    Xo, Yo, Zo = dy.shape[:3]
    xp = np.pad(x, ((p, p), (p, p), (p, p), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for ti, (a, bb, c) in enumerate(taps(k)):
        sl = xp[a:a + s * Xo:s, bb:bb + s * Yo:s, c:c + s * Zo:s, :]
        dW[ti] = np.einsum("xyzi,xyzo->io", sl, dy)
        dxp[a:a + s * Xo:s, bb:bb + s * Yo:s, c:c + s * Zo:s, :] += dy @ W[ti].T
    dx = dxp[p:p + X, p:p + Y, p:p + Z, :]
    db = dy.sum(axis=(0, 1, 2))
    return dx, dW, db


def up(x, W, b):
    """y[2v + t] = b + x[v] @ W[t] (2x2x2 stride-2 transposed convolution)."""
    X, Y, Z, _ = x.shape
    y = np.zeros((2 * X, 2 * Y, 2 * Z, W.shape[2]))
    for ti, (a, bb, c) in enumerate(taps(2)):
        y[a::2, bb::2, c::2, :] = x @ W[ti] + b
    return y


def up_backward(x, W, dy):
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for ti, (a, bb, c) in enumerate(taps(2)):
        g = dy[a::2, bb::2, c::2, :]
        dx += g @ W[ti].T
        dW[ti] = np.einsum("xyzi,xyzo->io", x, g)
    db = dy.sum(axis=(0, 1, 2))
    return dx, dW, db


def relu(x):
    return np.maximum(x, 0.0)


# ---------------------------------------------------------------- network
def layer_specs():
    """(name, kind, k, s, p, Ci, Co, relu) in execution order."""
    c0, c1, c2, c3 = CH
    L = []
    L += [("enc0a", "conv", 3, 1, 1, IN_CH, c0, True), ("enc0b", "conv", 3, 1, 1, c0, c0, True)]
    L += [("down0", "conv", 2, 2, 0, c0, c1, True)]
    L += [("enc1a", "conv", 3, 1, 1, c1, c1, True), ("enc1b", "conv", 3, 1, 1, c1, c1, True)]
    L += [("down1", "conv", 2, 2, 0, c1, c2, True)]
    L += [("enc2a", "conv", 3, 1, 1, c2, c2, True), ("enc2b", "conv", 3, 1, 1, c2, c2, True)]
    L += [("down2", "conv", 2, 2, 0, c2, c3, True)]
    L += [("bota", "conv", 3, 1, 1, c3, c3, True), ("botb", "conv", 3, 1, 1, c3, c3, True)]
    L += [("up2", "up", 2, 2, 0, c3, c2, True)]
    L += [("dec2a", "conv", 3, 1, 1, 2 * c2, c2, True), ("dec2b", "conv", 3, 1, 1, c2, c2, True)]
    L += [("up1", "up", 2, 2, 0, c2, c1, True)]
    L += [("dec1a", "conv", 3, 1, 1, 2 * c1, c1, True), ("dec1b", "conv", 3, 1, 1, c1, c1, True)]
    L += [("up0", "up", 2, 2, 0, c1, c0, True)]
    L += [("dec0a", "conv", 3, 1, 1, 2 * c0, c0, True), ("dec0b", "conv", 3, 1, 1, c0, c0, True)]
    L += [("out", "conv", 1, 1, 0, c0, OUT_CH, False)]
    return L


def param_layout():
    """Flat FP32 parameter vector: for each layer W [k^3, Ci, Co] then b [Co]."""
    off, out = 0, {}
    for name, kind, k, s, p, ci, co, act in layer_specs():
        nW = k ** 3 * ci * co
        out[name] = (off, off + nW, off + nW + co)
        off += nW + co
    return out, off


def unpack(params):
    lay, _ = param_layout()
    res = {}
    for name, kind, k, s, p, ci, co, act in layer_specs():
        a, bw, e = lay[name]
        res[name] = (params[a:bw].reshape(k ** 3, ci, co), params[bw:e])
    return res


def init_params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    lay, n = param_layout()
    params = np.zeros(n)
    for name, kind, k, s, p, ci, co, act in layer_specs():
        a, bw, e = lay[name]
        fan_in = k ** 3 * ci if kind == "conv" else ci
        params[a:bw] = rng.normal(0.0, scale * np.sqrt(2.0 / fan_in), bw - a)
    return params


def _ident(a):
    return a


def forward(params, x, keep=False, rnd=_ident):
    """U-Net forward; x [X,Y,Z,IN_CH] with X, Y, Z multiples of 8.

    ``rnd`` is applied to every stored layer output (identity by default; the
    BF16 precision model passes :func:`bf16`, mirroring where the MFMA kernels
    store BF16 activations; the arithmetic itself stays FP64)."""
    P = unpack(params)
    spec = {s[0]: s for s in layer_specs()}
    acts = {"x": x}

    def run(name, inp):
        _, kind, k, s, p, ci, co, act = spec[name]
        W, b = P[name]
        y = conv(inp, W, b, k, s, p) if kind == "conv" else up(inp, W, b)
        if act:
            y = relu(y)
        y = rnd(y)
        acts[name + ":in"] = inp
        acts[name] = y
        return y

    h = run("enc0b", run("enc0a", x))
    s0 = h
    h = run("enc1b", run("enc1a", run("down0", h)))
    s1 = h
    h = run("enc2b", run("enc2a", run("down1", h)))
    s2 = h
    h = run("botb", run("bota", run("down2", h)))
    h = np.concatenate([run("up2", h), s2], axis=-1)
    h = run("dec2b", run("dec2a", h))
    h = np.concatenate([run("up1", h), s1], axis=-1)
    h = run("dec1b", run("dec1a", h))
    h = np.concatenate([run("up0", h), s0], axis=-1)
    h = run("dec0b", run("dec0a", h))
    y = run("out", h)
    return (y, acts) if keep else y


def backward(params, x, dy, rnd=_ident):
    """Parameter gradient of <dy, forward(params, x)> (flat, like params).

    ``rnd`` is applied to every stored activation and activation gradient
    (see :func:`forward`)."""
    P = unpack(params)
    spec = {s[0]: s for s in layer_specs()}
    y, acts = forward(params, x, keep=True, rnd=rnd)
    lay, n = param_layout()
    grad = np.zeros(n)

    def back(name, g):
        _, kind, k, s, p, ci, co, act = spec[name]
        W, b = P[name]
        if act:
            g = g * (acts[name] > 0)
        inp = acts[name + ":in"]
        if kind == "conv":
            dx, dW, db = conv_backward(inp, W, g, k, s, p)
        else:
            dx, dW, db = up_backward(inp, W, g)
        a, bw, e = lay[name]
        grad[a:bw] += dW.ravel()
        grad[bw:e] += db
        return rnd(dx)

    c0, c1, c2, _ = CH
    g = back("out", dy)
    g = back("dec0a", back("dec0b", g))
    gs0 = g[..., c0:]
    g = back("up0", g[..., :c0])
    g = back("dec1a", back("dec1b", g))
    gs1 = g[..., c1:]
    g = back("up1", g[..., :c1])
    g = back("dec2a", back("dec2b", g))
    gs2 = g[..., c2:]
    g = back("up2", g[..., :c2])
    g = back("down2", back("bota", back("botb", g)))
    g = back("down1", back("enc2a", back("enc2b", rnd(g + gs2))))
    g = back("down0", back("enc1a", back("enc1b", rnd(g + gs1))))
    back("enc0a", back("enc0b", rnd(g + gs0)))
    return grad


def loss(y, target, mask):
    """Masked relative L2 on the first 3 output channels: |m (y - t)|^2 / |m t|^2."""
    d = (y[..., :3] - target[..., :3]) * mask[..., None]
    den = np.sum((target[..., :3] * mask[..., None]) ** 2)
    return np.sum(d * d) / den


def loss_grad(y, target, mask):
    den = np.sum((target[..., :3] * mask[..., None]) ** 2)
    g = np.zeros_like(y)
    g[..., :3] = 2.0 * (y[..., :3] - target[..., :3]) * (mask[..., None] ** 2) / den
    return g


def bf16(a):
    """Round to bfloat16 (round to nearest even) and back to float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)

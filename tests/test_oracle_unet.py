"""Pins of the network oracle (oracle/unet.py): convolutions against scipy's
correlation, the transposed convolution against an explicit scatter loop,
and the hand-derived backward pass against central finite differences."""
import numpy as np
import scipy.signal

from oracle import unet as U


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(6, 5, 7, 1))
    W = rng.normal(size=(27, 1, 1))
    y = U.conv(x, W, np.zeros(1), 3, 1, 1)
    ref = scipy.signal.correlate(x[..., 0], W[:, 0, 0].reshape(3, 3, 3), mode="same")
    assert np.allclose(y[..., 0], ref, atol=1e-12)
    # multi-channel: sum over input channels of single-channel correlations
    x = rng.normal(size=(6, 6, 6, 3))
    W = rng.normal(size=(27, 3, 2))
    y = U.conv(x, W, np.array([0.5, -1.0]), 3, 1, 1)
    for o in range(2):
        ref = sum(scipy.signal.correlate(x[..., i], W[:, i, o].reshape(3, 3, 3), mode="same")
                  for i in range(3)) + [0.5, -1.0][o]
        assert np.allclose(y[..., o], ref, atol=1e-12)


def test_strided_conv_and_transposed_conv_definitions():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(4, 6, 8, 3))
    W = rng.normal(size=(8, 3, 2))
    y = U.conv(x, W, np.zeros(2), 2, 2, 0)
    assert y.shape == (2, 3, 4, 2)
    i, j, k = 1, 2, 3
    ref = sum(x[2 * i + a, 2 * j + b, 2 * k + c] @ W[(a * 2 + b) * 2 + c]
              for a in range(2) for b in range(2) for c in range(2))
    assert np.allclose(y[i, j, k], ref)
    xs = rng.normal(size=(2, 3, 4, 3))
    Wu = rng.normal(size=(8, 3, 5))
    bu = rng.normal(size=5)
    yu = U.up(xs, Wu, bu)
    ref = np.zeros((4, 6, 8, 5))
    for i in range(2):
        for j in range(3):
            for k in range(4):
                for t, (a, b, c) in enumerate(U.taps(2)):
                    ref[2 * i + a, 2 * j + b, 2 * k + c] = xs[i, j, k] @ Wu[t] + bu
    assert np.allclose(yu, ref)


def test_layer_adjoints():
    """<conv(x), g> = <x, conv^T(g)> and the weight gradients are exact."""
    rng = np.random.default_rng(2)
    for k, s, p in ((3, 1, 1), (2, 2, 0), (1, 1, 0)):
        x = rng.normal(size=(4, 4, 6, 3))
        W = rng.normal(size=(k ** 3, 3, 2))
        b = rng.normal(size=2)
        y = U.conv(x, W, b, k, s, p)
        g = rng.normal(size=y.shape)
        dx, dW, db = U.conv_backward(x, W, g, k, s, p)
        assert np.isclose(np.sum((y - b) * g), np.sum(x * dx))
        assert np.isclose(np.sum((y - b) * g), np.sum(W * dW))
        assert np.allclose(db, g.sum(axis=(0, 1, 2)))
    x = rng.normal(size=(2, 3, 2, 4))
    W = rng.normal(size=(8, 4, 3))
    y = U.up(x, W, np.zeros(3))
    g = rng.normal(size=y.shape)
    dx, dW, db = U.up_backward(x, W, g)
    assert np.isclose(np.sum(y * g), np.sum(x * dx))
    assert np.isclose(np.sum(y * g), np.sum(W * dW))


def test_unet_backward_matches_finite_differences():
    rng = np.random.default_rng(3)
    params = U.init_params(seed=4)
    params += 0.01 * rng.normal(size=params.shape)  # nonzero biases
    x = rng.normal(size=(8, 8, 16, U.IN_CH))
    y = U.forward(params, x)
    assert y.shape == (8, 8, 16, U.OUT_CH)
    dy = rng.normal(size=y.shape)
    grad = U.backward(params, x, dy)
    lay, _ = U.param_layout()
    for name, (a, b, e) in lay.items():
        d = np.zeros_like(params)
        d[a:e] = rng.normal(size=e - a)
        # the network is piecewise linear: a small step perturbing one layer at
        # a time stays inside one ReLU activation pattern
        h = 1e-7
        fp = np.sum(U.forward(params + h * d, x) * dy)
        fm = np.sum(U.forward(params - h * d, x) * dy)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - grad @ d) <= 1e-6 * max(1.0, abs(fd)), name


def test_loss_gradient():
    rng = np.random.default_rng(5)
    y = rng.normal(size=(4, 4, 4, U.OUT_CH))
    t = rng.normal(size=y.shape)
    m = (rng.random(size=(4, 4, 4)) > 0.3).astype(float)
    g = U.loss_grad(y, t, m)
    d = rng.normal(size=y.shape)
    h = 1e-6
    fd = (U.loss(y + h * d, t, m) - U.loss(y - h * d, t, m)) / (2 * h)
    assert abs(fd - np.sum(g * d)) <= 1e-7 * max(1.0, abs(fd))
    assert np.all(g[..., 3:] == 0)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 3.14159, -2.5e-3])
    r = U.bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7
    assert np.all(np.abs(r - vals) <= 2 ** -8 * np.abs(vals))

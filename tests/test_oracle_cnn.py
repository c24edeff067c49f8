"""Pins of the FP64 window-network oracle: finite differences and layer identities (no GPU)."""
import numpy as np
import pytest

from oracle import cnn


def small_batch(n=3, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, 6, 16, 16)), rng.standard_normal((n, 3))


def test_param_count():
    assert cnn.COUNT == 864 + 16 + 4608 + 32 + 64 * 2048 + 64 + 192 + 3


def test_conv_matches_direct_sum():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 5))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    for stride in (1, 2):
        y = cnn.conv2d(x, W, b, stride)
        xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
        for n in range(2):
            for o in range(4):
                for i in range(y.shape[2]):
                    for j in range(y.shape[3]):
                        ref = b[o] + np.sum(W[o] * xp[n, :, i * stride:i * stride + 3,
                                                    j * stride:j * stride + 3])
                        assert abs(y[n, o, i, j] - ref) < 1e-12


def test_gradient_by_finite_differences():
    x, t = small_batch()
    theta = cnn.init_params(3) * 0.5 + 0.01
    loss, g = cnn.loss_and_grad(theta, x, t)
    rng = np.random.default_rng(7)
    offsets = np.cumsum([0] + [int(np.prod(s)) for _, s in cnn.SHAPES])
    idx = []
    for a, b in zip(offsets[:-1], offsets[1:]):          # a few entries of every tensor
        idx += list(rng.integers(a, b, size=4))
    for i in idx:
        h = 1e-6
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (cnn.loss_and_grad(tp, x, t)[0] - cnn.loss_and_grad(tm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_directional_derivative():
    x, t = small_batch(4, 2)
    theta = cnn.init_params(5)
    loss, g = cnn.loss_and_grad(theta, x, t)
    v = np.random.default_rng(9).standard_normal(theta.shape)
    h = 1e-6
    fd = (cnn.loss_and_grad(theta + h * v, x, t)[0] - cnn.loss_and_grad(theta - h * v, x, t)[0]) / (2 * h)
    assert fd == pytest.approx(g @ v, rel=1e-6)


def test_features_layout_and_degree_label():
    f = np.arange(2 * 3 * 4 * 4).reshape(2, 3, 4, 4) * (1 + 2j)
    x = cnn.window_features(f)
    assert x.shape == (2, 6, 4, 4)
    np.testing.assert_array_equal(x[:, 2], f[:, 1].real)
    np.testing.assert_array_equal(x[:, 5], f[:, 2].imag)
    assert cnn.degree_label(100.0, 200.0, 1e4) == pytest.approx(np.ceil(np.arccosh(1e4) / np.arccosh(1 + 2 * 100 / 9800)))
    assert cnn.degree_label(1000.0, 1000.5, 1e7) == 128.0

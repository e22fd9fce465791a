"""Pins of the warm-start network oracle against independent definitions."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn


def dilated(K, d):
    out = np.zeros((2 * d + 1, 2 * d + 1))
    out[::d, ::d] = K
    return out


@pytest.mark.parametrize("dil", [1, 2, 4, 8])
def test_conv_matches_scipy_correlate(dil):
    rng = np.random.default_rng(dil)
    x = rng.standard_normal((2, 3, 13, 11))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    out = cnn.conv2d(x, W, b, dil)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate2d(x[n, c], dilated(W[o, c], dil), mode="same")
                             for c in range(3))
            np.testing.assert_allclose(out[n, o], ref, rtol=1e-12, atol=1e-12)


def test_param_count_and_layout():
    assert cnn.param_count() == 2 * 32 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 32 * 2 * 9 + 2
    th = np.arange(cnn.param_count(), dtype=float)
    parts = cnn.unpack(th)
    assert parts[0][0].shape == (32, 2, 3, 3) and parts[3][1].shape == (2,)
    assert parts[1][0][0, 0, 0, 0] == 2 * 32 * 9 + 32       # W2 follows b1


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    th = cnn.init_params(1) + 0.01 * rng.standard_normal(cnn.param_count())
    x = rng.uniform(0, 2, (2, 2, 9, 9))
    t = rng.standard_normal((2, 2, 9, 9))
    loss, g = cnn.grad(th, x, t)
    assert loss == pytest.approx(cnn.mse(cnn.forward(th, x)[-1], t))
    # every layer's weights and biases
    offs, off = [], 0
    for ci, co, _, _ in cnn.LAYERS:
        offs += list(rng.integers(off, off + co * ci * 9, 12)) + list(off + co * ci * 9 + np.arange(min(co, 3)))
        off += co * ci * 9 + co
    h = 1e-6
    for k in offs:
        e = np.zeros_like(th)
        e[k] = h
        fd = (cnn.mse(cnn.forward(th + e, x)[-1], t) - cnn.mse(cnn.forward(th - e, x)[-1], t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (k, fd, g[k])


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = cnn.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01, eps=0.0)
    np.testing.assert_allclose(th, -0.01 * np.sign(g), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_zero_weights_output_is_last_bias():
    th = np.zeros(cnn.param_count())
    th[-2:] = [0.25, -4.0]
    out = cnn.forward(th, np.ones((1, 2, 8, 8)))[-1]
    assert np.all(out[0, 0] == 0.25) and np.all(out[0, 1] == -4.0)


@pytest.mark.parametrize("side", [8, 13, 32, 64, 256])
def test_network_input_preserves_mass(side):
    rng = np.random.default_rng(side)
    a = rng.uniform(0, 1, side * side)
    a /= a.sum()
    b = rng.uniform(0, 1, side * side)
    b /= b.sum()
    x = cnn.network_input(a, b, side)
    assert x.shape == (2, 32, 32)
    assert x[0].sum() / 32 ** 2 == pytest.approx(1.0, rel=1e-12)
    assert x[1].sum() / 32 ** 2 == pytest.approx(1.0, rel=1e-12)
    if side == 32:
        np.testing.assert_allclose(x[0], a.reshape(32, 32) * 1024, rtol=1e-14)
    if side == 256:
        pooled = a.reshape(32, 8, 32, 8).sum(axis=(1, 3)) * 1024
        np.testing.assert_allclose(x[0], pooled, rtol=1e-12)


def test_upsample_identity_and_constants():
    rng = np.random.default_rng(3)
    P = rng.standard_normal((2, 32, 32))
    y, z = cnn.upsample_duals(P, 32)
    np.testing.assert_allclose(y, P[0].reshape(-1) * 1024, rtol=1e-14)
    np.testing.assert_allclose(z, P[1].reshape(-1) * 1024, rtol=1e-14)
    C = np.full((2, 32, 32), 0.5)
    y, z = cnn.upsample_duals(C, 20)
    np.testing.assert_allclose(y, 0.5 * 400, rtol=1e-14)
    # a linear ramp is reproduced exactly away from the border
    R = np.stack([np.add.outer(np.arange(32.0), np.zeros(32))] * 2)
    y, _ = cnn.upsample_duals(R, 64)
    rows = ((np.arange(64) + 0.5) * 0.5 - 0.5)
    inner = (rows >= 0) & (rows <= 31)
    np.testing.assert_allclose(y.reshape(64, 64)[inner, 0], rows[inner] * 4096, rtol=1e-12)


def test_dual_targets_gauge():
    rng = np.random.default_rng(4)
    y, z = rng.standard_normal(64), rng.standard_normal(64)
    t = cnn.dual_targets(y, z, 8)
    assert t[0].mean() == pytest.approx(t[1].mean(), abs=1e-15)
    # y_i + z_j unchanged up to the side^2 scale
    np.testing.assert_allclose(t[0].reshape(-1)[3] + t[1].reshape(-1)[5], (y[3] + z[5]) / 64)

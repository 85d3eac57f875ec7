"""Pins of the numpy reference network (oracle/unet.py) against things other than itself:
library cross-correlation, adjoint identities, central finite differences of the loss,
a zero network, and the closed form of Adam under a constant gradient."""
import numpy as np
import pytest
from scipy import signal

from oracle import unet


def test_conv_matches_library_correlation():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((9, 12, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    Y = unet.conv(X, W, b)
    for o in range(4):
        ref = b[o] + sum(signal.correlate2d(X[:, :, c], W[o, :, :, c], mode="same", boundary="fill")
                         for c in range(3))
        np.testing.assert_allclose(Y[:, :, o], ref, rtol=1e-12, atol=1e-12)
    W1 = rng.standard_normal((5, 1, 1, 3))
    np.testing.assert_allclose(unet.conv(X, W1, np.zeros(5)), X @ W1[:, 0, 0, :].T, rtol=1e-13)


@pytest.mark.parametrize("k", [1, 3])
def test_conv_adjoints(k):
    rng = np.random.default_rng(1)
    X = rng.standard_normal((8, 6, 5))
    W = rng.standard_normal((7, k, k, 5))
    dY = rng.standard_normal((8, 6, 7))
    dX, dW, db = unet.conv_backward(X, W, dY)
    lhs = np.sum(dY * unet.conv(X, W, np.zeros(7)))
    assert abs(lhs - np.sum(X * dX)) <= 1e-11 * abs(lhs) + 1e-11
    assert abs(lhs - np.sum(W * dW)) <= 1e-11 * abs(lhs) + 1e-11
    np.testing.assert_allclose(db, dY.sum(axis=(0, 1)), rtol=1e-14)


def test_pool_up_adjoints():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((8, 12, 3))
    Y = rng.standard_normal((4, 6, 3))
    assert abs(np.sum(unet.pool(X) * Y) - np.sum(X * unet.pool_backward(Y))) <= 1e-12
    assert abs(np.sum(unet.up(Y) * X) - np.sum(Y * unet.up_backward(X))) <= 1e-12
    np.testing.assert_allclose(unet.pool(unet.up(Y)), Y, rtol=1e-15)


def _small_problem(seed=3, H=8, c_in=7, c_out=4):
    rng = np.random.default_rng(seed)
    theta = unet.he_init(c_in, c_out, rng)
    theta[-c_out:] = rng.standard_normal(c_out) * 0.1
    x = rng.standard_normal((H, H, c_in))
    t = rng.standard_normal((H, H, c_out))
    return rng, theta, x, t


def test_loss_gradient_finite_differences():
    rng, theta, x, t = _small_problem()
    L, g, gx = unet.loss_and_grad(theta, x, t)
    assert g.shape == theta.shape and gx.shape == x.shape
    # parameters from every layer (weights and biases), central differences
    offs = np.cumsum([0] + [co * k * k * ci + co for _, k, ci, co in unet.layers(7, 4)])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):
        idx += list(rng.integers(a, b, 4)) + [b - 1]
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (unet.loss(unet.forward(tp, x, 4), t) - unet.loss(unet.forward(tm, x, 4), t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])
    for _ in range(12):
        p = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[p] += h
        xm[p] -= h
        fd = (unet.loss(unet.forward(theta, xp, 4), t) - unet.loss(unet.forward(theta, xm, 4), t)) / (2 * h)
        assert abs(fd - gx[p]) <= 1e-6 * max(abs(gx[p]), 1e-3), (p, fd, gx[p])


def test_zero_network_outputs_head_bias():
    c_in, c_out = 7, 4
    theta = np.zeros(unet.num_params(c_in, c_out))
    theta[-c_out:] = [1.0, -2.0, 0.5, 3.0]
    y = unet.forward(theta, np.random.default_rng(4).standard_normal((8, 8, c_in)), c_out)
    np.testing.assert_array_equal(y, np.broadcast_to([1.0, -2.0, 0.5, 3.0], y.shape))


def test_adam_constant_gradient_closed_form():
    # with a constant gradient g, m̂ = g and v̂ = g² after bias correction, so every step
    # moves each parameter by lr·g/(|g|+ε)
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    th = theta.copy()
    for t in range(1, 6):
        th, m, v = unet.adam_step(th, m, v, g, t, lr=1e-2)
        np.testing.assert_allclose(th, theta - t * 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-14)


def test_pack_unpack_round_trip():
    rng = np.random.default_rng(6)
    Q, n = 3, 9
    r = rng.standard_normal(Q * n * n) + 1j * rng.standard_normal(Q * n * n)
    kf = rng.standard_normal((2, n * n))
    x = unet.pack_input(r, kf, 4.0, Q, n)
    H = unet.padded_size(n)
    assert x.shape == (H, H, 2 * Q + 2) and H == 12
    np.testing.assert_allclose(np.sum(x[:, :, :2 * Q] ** 2), Q * n * n, rtol=1e-13)
    assert np.all(x[n:, :, :] == 0) and np.all(x[:, n:, :] == 0)
    np.testing.assert_allclose(x[2, 5, 2 * Q + 1], kf[1, 2 * n + 5] / 4.0, rtol=1e-15)
    # channel 2q+1 of pixel (y, x) is Im r_q(x, y) up to the scaling
    s = np.sqrt(Q * n * n) / np.linalg.norm(r)
    np.testing.assert_allclose(x[4, 7, 2 * 1 + 1], r[1 * n * n + 4 * n + 7].imag * s, rtol=1e-13)
    c = rng.standard_normal(Q * n * n) + 1j * rng.standard_normal(Q * n * n)
    np.testing.assert_allclose(unet.unpack_output(unet.pack_target(c, 2.5, Q, n), 2.5, Q, n), c, rtol=1e-13)


def test_bf16_round_exact_values():
    # representable values are fixed points; halfway cases go to the even significand;
    # the relative rounding error is at most the unit roundoff 2^-8 of an 8-bit significand
    vals = np.array([1.0, -2.0, 0.0, 1.0 + 2 ** -7, 3.0 * 2 ** -130, 65280.0])
    np.testing.assert_array_equal(unet.bf16_round(vals), vals)
    assert unet.bf16_round(1.0 + 2 ** -8) == 1.0                    # tie, even neighbour 1.0
    assert unet.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6      # tie, even neighbour 1+2^-6
    assert unet.bf16_round(1.0 + 2 ** -8 + 2 ** -20) == 1.0 + 2 ** -7
    assert unet.bf16_round(-(1.0 + 2 ** -8 + 2 ** -20)) == -(1.0 + 2 ** -7)
    x = np.random.default_rng(7).standard_normal(10000) * 10.0 ** np.random.default_rng(8).integers(-20, 20, 10000)
    r = unet.bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-4))
    assert np.max(np.abs(r - x) / np.abs(x)) > 2.0 ** -9          # and the bound is attained
    # the bfloat16 grid: 8 significant bits
    m, _ = np.frexp(r)
    assert np.all((m * 2 ** 8) == np.round(m * 2 ** 8))


def test_rounded_network_is_the_exact_one_on_bf16_data():
    # with data already on the bfloat16 grid and rounding that changes nothing, the rounded
    # forward pass equals the exact one; with real rounding it stays close
    rng, theta, x, t = _small_problem(seed=11)
    y0 = unet.forward(theta, x, 4)
    y1 = unet.forward(theta, x, 4, rnd=lambda a: a)
    np.testing.assert_array_equal(y0, y1)
    y2 = unet.forward(theta, x, 4, rnd=unet.bf16_round)
    assert np.linalg.norm(y2 - y0) <= 2e-2 * np.linalg.norm(y0)
    L, g, _ = unet.loss_and_grad(theta, x, t, rnd=unet.bf16_round)
    L0, g0, _ = unet.loss_and_grad(theta, x, t)
    assert abs(L - L0) <= 1e-2 * L0

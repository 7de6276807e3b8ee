"""Pins of the closure oracle (CPU only): brute-force convolution, central
finite-difference gradients, box-filter invariants and Fourier transfer,
GELU identities, and Adam against its first-step closed form."""
import math

import numpy as np
import pytest

from oracle import closure as C


def _brute_conv(x, W, b):
    cin, nz, ny, nx = x.shape
    cout = W.shape[0]
    y = np.zeros((cout, nz, ny, nx))
    for o in range(cout):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    acc = b[o]
                    for t, (dz, dy, dx) in enumerate(C.TAPS):
                        for c in range(cin):
                            acc += W[o, t, c] * x[c, (k + dz) % nz, (j + dy) % ny, (i + dx) % nx]
                    y[o, k, j, i] = acc
    return y


def test_conv_matches_brute_force():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 4, 3, 5))
    W = rng.standard_normal((2, 27, 3))
    b = rng.standard_normal(2)
    assert np.allclose(C.conv3d(x, W, b), _brute_conv(x, W, b), rtol=1e-13, atol=1e-13)


def test_delta_kernel_is_a_shift():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 5, 6, 7))
    for t, (dz, dy, dx) in enumerate(C.TAPS):
        W = np.zeros((2, 27, 2))
        W[0, t, 0] = W[1, t, 1] = 1.0
        y = C.conv3d(x, W, np.zeros(2))
        # y[c, k, j, i] = x[c, k+dz, j+dy, i+dx]
        assert y[0, 1, 2, 3] == x[0, (1 + dz) % 5, (2 + dy) % 6, (3 + dx) % 7]
        assert np.array_equal(y[1], np.roll(x[1], (-dz, -dy, -dx), axis=(0, 1, 2)))


def test_network_gradients_by_central_differences():
    rng = np.random.default_rng(3)
    n = 4
    params = C.init_params(7)
    x = rng.standard_normal((8, n, n, n))
    target = rng.standard_normal((8, n, n, n))

    def loss(ps, xx):
        return C.mse(C.forward(ps, xx)[0], target)

    y, cache = C.forward(params, x)
    grads, dx = C.backward(params, cache, C.mse_grad(y, target))
    h = 1e-6
    for li in range(3):
        W, b = params[li]
        for idx in [(0, 0, 0), (5, 13, 3), (W.shape[0] - 1, 26, W.shape[2] - 1)]:
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            pp = [p if i != li else (Wp, b) for i, p in enumerate(params)]
            pm = [p if i != li else (Wm, b) for i, p in enumerate(params)]
            fd = (loss(pp, x) - loss(pm, x)) / (2 * h)
            assert grads[li][0][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)
        bp, bm = b.copy(), b.copy()
        bp[1] += h
        bm[1] -= h
        fd = (loss([p if i != li else (W, bp) for i, p in enumerate(params)], x) -
              loss([p if i != li else (W, bm) for i, p in enumerate(params)], x)) / (2 * h)
        assert grads[li][1][1] == pytest.approx(fd, rel=1e-6, abs=1e-10)
    for idx in [(0, 0, 0, 0), (7, 3, 2, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (loss(params, xp) - loss(params, xm)) / (2 * h)
        assert dx[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_box_filter_invariants_and_transfer():
    rng = np.random.default_rng(4)
    f = rng.standard_normal((2, 16, 12, 8))
    c = C.box_filter4(f)
    assert c.shape == (2, 4, 3, 2)
    assert np.allclose(64 * c.sum(axis=(1, 2, 3)), f.sum(axis=(1, 2, 3)), rtol=1e-14, atol=1e-12)
    assert np.allclose(C.box_filter4(np.full((8, 8, 8), 3.25)), 3.25)
    # a mode cos(k x) on the fine grid (h = 2 pi / N) filters to
    # A(k) cos(k (x_c + 1.5 h)) on the block corners x_c = 4 I h, with
    # A(k) = sin(2 k h) / (4 sin(k h / 2))
    N, k = 32, 3
    h = 2 * math.pi / N
    x = np.arange(N) * h
    f1 = np.broadcast_to(np.cos(k * x), (4, 4, N)).copy()
    cf = C.box_filter4(f1)[0, 0]
    A = math.sin(2 * k * h) / (4 * math.sin(k * h / 2))
    xc = np.arange(N // 4) * 4 * h
    assert np.allclose(cf, A * np.cos(k * (xc + 1.5 * h)), rtol=0, atol=1e-14)


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    g = C.gelu(x)
    assert np.allclose(g - C.gelu(-x), x, atol=1e-14)  # x Phi(x) + x Phi(-x) = x
    assert C.gelu(0.0) == 0.0 and C.gelu_grad(0.0) == 0.5
    assert abs(C.gelu(8.0) - 8.0) < 1e-12
    h = 1e-6
    assert np.allclose(C.gelu_grad(x), (C.gelu(x + h) - C.gelu(x - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = C.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # step 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)

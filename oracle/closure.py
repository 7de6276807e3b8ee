"""FP64 oracle of the learned closure (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the CPU-baseline leg of the benchmark use
this module; the HIP closure kernels never import it.

The closure is not in the paper (its discussion names machine-learned
reconstruction of turbulent flow only as related work, Section 6).  What is
computed here is the plain definition of each piece:

* ``box_filter4``: coarse[I,J,K] = mean of fine[4I+a, 4J+b, 4K+c], a,b,c in 0..3.
* ``conv3d``: periodic ("circular") 3x3x3 convolution,
  y[o, p] = b[o] + sum_{t, c} W[o, t, c] x[c, p + off(t)], with tap
  t = 9 (dz+1) + 3 (dy+1) + (dx+1) for offsets dz, dy, dx in {-1, 0, 1}.
* ``gelu``: x * Phi(x) = x (1 + erf(x / sqrt 2)) / 2 (the exact form).
* the network: conv 8->32, GELU, conv 32->32, GELU, conv 32->8.
* ``mse``: mean of squared differences over every element.
* ``adam``: Kingma & Ba with bias correction.

Arrays are channel-first float64: x has shape (C, nz, ny, nx); weights
(Cout, 27, Cin); biases (Cout,).
"""
from __future__ import annotations

import math

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
LAYERS = ((8, 32, True), (32, 32, True), (32, 8, False))  # (cin, cout, gelu)


def box_filter4(fine: np.ndarray) -> np.ndarray:
    """Mean over 4x4x4 blocks of the last three axes."""
    *lead, nz, ny, nx = fine.shape
    assert nz % 4 == 0 and ny % 4 == 0 and nx % 4 == 0
    r = np.asarray(fine, dtype=np.float64).reshape(*lead, nz // 4, 4, ny // 4, 4, nx // 4, 4)
    return r.mean(axis=(-5, -3, -1))


def shifted(x: np.ndarray, tap) -> np.ndarray:
    """s[c, p] = x[c, p + off(tap)] with periodic wrap."""
    dz, dy, dx = tap
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


def conv3d(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    cout = W.shape[0]
    y = np.empty((cout,) + x.shape[1:])
    y[:] = b[:, None, None, None]
    for t, tap in enumerate(TAPS):
        y += np.einsum("oc,czyx->ozyx", W[:, t, :], shifted(x, tap))
    return y


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def init_params(seed: int):
    """He-style initial weights (the GPU training uses the same recipe)."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout, _ in LAYERS:
        std = math.sqrt(2.0 / (27 * cin))
        params.append((rng.standard_normal((cout, 27, cin)) * std, np.zeros(cout)))
    return params


def forward(params, x):
    """Returns (y, cache); cache keeps each layer's input and pre-activation."""
    cache = []
    h = x
    for (W, b), (_, _, act) in zip(params, LAYERS):
        z = conv3d(h, W, b)
        cache.append((h, z))
        h = gelu(z) if act else z
    return h, cache


def conv3d_backward(x, W, dz):
    """Gradients of y = conv3d(x, W, b) given dL/dy = dz."""
    dW = np.empty_like(W)
    for t, tap in enumerate(TAPS):
        dW[:, t, :] = np.einsum("ozyx,czyx->oc", dz, shifted(x, tap))
    db = dz.sum(axis=(1, 2, 3))
    dx = np.zeros_like(x)
    for t, (tz, ty, tx) in enumerate(TAPS):
        dx += np.einsum("oc,ozyx->czyx", W[:, t, :], shifted(dz, (-tz, -ty, -tx)))
    return dW, db, dx


def backward(params, cache, dy):
    grads = [None] * len(params)
    g = dy
    for i in reversed(range(len(params))):
        W, _ = params[i]
        h, z = cache[i]
        dz = g * gelu_grad(z) if LAYERS[i][2] else g
        dW, db, dh = conv3d_backward(h, W, dz)
        grads[i] = (dW, db)
        g = dh
    return grads, g


def mse(y, target) -> float:
    d = np.asarray(y, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d))


def mse_grad(y, target):
    d = np.asarray(y, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return 2.0 * d / d.size


def adam(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** t)
    vhat = v / (1 - b2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v

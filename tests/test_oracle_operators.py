"""Pins of the oracle's finite-difference operators (CPU only).

Each check ties the oracle to something other than itself:
* the weights come out of an exact rational solve of the Taylor system for
  the central stencil of order k = 2r, r = 1..4 (Section 4, Eq. stencil-fd),
  and for r = 3 equal the printed sixth-order integers;
* on any Fourier mode each operator acts as multiplication by its discrete
  symbol, a closed form in sines/cosines of k*h (exact to roundoff);
* the error against the analytic derivative falls by 2^(2r) per grid
  doubling;
* periodic sums of every operator vanish and div(curl A) vanishes (the
  one-dimensional operators along different axes commute).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

TWO_PI = 2 * math.pi


ORDERS = (2, 4, 6, 8)


def _taylor_weights(deriv_order: int, r: int = 3):
    """Exact weights w_m (m = -r..r) with sum_m w_m m^p = p! [p == order],
    p = 0..2r: the unique central stencil of order 2r on 2r+1 points."""
    offs = list(range(-r, r + 1))
    n = len(offs)
    A = [[Fraction(m) ** p for m in offs] for p in range(n)]
    b = [Fraction(math.factorial(p)) if p == deriv_order else Fraction(0) for p in range(n)]
    # Gauss-Jordan on fractions
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        pv = M[c][c]
        M[c] = [v / pv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                fac = M[r][c]
                M[r] = [a - fac * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def test_taylor_solve_gives_the_sixth_order_integers():
    assert _taylor_weights(1) == [Fraction(x, 60) for x in (-1, 9, -45, 0, 45, -9, 1)]
    assert _taylor_weights(2) == [Fraction(x, 180) for x in (2, -27, 270, -490, 270, -27, 2)]


@pytest.mark.parametrize("order", ORDERS)
def test_weights_match_exact_taylor_solve(oracle_mod, order):
    r = order // 2
    a1, a2 = oracle_mod.weights(order)
    assert len(a1) == len(a2) == 2 * r + 1
    for got, exact in zip(a1, _taylor_weights(1, r)):
        assert got == float(exact)
    for got, exact in zip(a2, _taylor_weights(2, r)):
        assert got == float(exact)


def test_bad_order_rejected(oracle_mod):
    with pytest.raises(ValueError):
        oracle_mod.weights(5)
    with pytest.raises(ValueError):
        oracle_mod.deriv(np.zeros((4, 4, 4)), "d1x", order=10)


def _grid(n, lengths=(TWO_PI,) * 3):
    nx, ny, nz = n
    x = np.arange(nx) * lengths[0] / nx
    y = np.arange(ny) * lengths[1] / ny
    z = np.arange(nz) * lengths[2] / nz
    return np.meshgrid(z, y, x, indexing="ij")[::-1]  # X, Y, Z each (nz, ny, nx)


def _k_tilde(theta, h):
    return (45 * np.sin(theta) - 9 * np.sin(2 * theta) + np.sin(3 * theta)) / (30 * h)


def _beta(theta):
    """Symbol of the second-derivative weights at unit step: sum_m b_m e^{i m theta}."""
    return (-490 + 540 * np.cos(theta) - 54 * np.cos(2 * theta) + 4 * np.cos(3 * theta)) / 180


def _symbols(order):
    """(k_tilde, beta) of the stencil of this order: the printed sixth-order
    closed forms, else the sums over the exact Taylor weights."""
    if order == 6:
        return _k_tilde, _beta
    r = order // 2
    w1 = [float(x) for x in _taylor_weights(1, r)]
    w2 = [float(x) for x in _taylor_weights(2, r)]
    k_t = lambda th, h: sum(w * np.sin(m * th) for m, w in zip(range(-r, r + 1), w1)) / h
    beta = lambda th: sum(w * np.cos(m * th) for m, w in zip(range(-r, r + 1), w2))
    return k_t, beta


MODES = [(1, 0, 0), (2, -1, 3), (-3, 2, 1), (5, 4, -2), (0, 0, 6)]


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("kvec", MODES)
def test_fourier_symbols_exact(oracle_mod, kvec, order):
    k_tilde, beta = _symbols(order)
    n = (16, 12, 14)
    L = (TWO_PI, 1.5 * TWO_PI, 0.75 * TWO_PI)
    X, Y, Z = _grid(n, L)
    h = [L[a] / n[a] for a in range(3)]
    kk = [TWO_PI * kvec[a] / L[a] for a in range(3)]
    phase = kk[0] * X + kk[1] * Y + kk[2] * Z + 0.3
    f = np.cos(phase)
    s = np.sin(phase)
    th = [kk[a] * h[a] for a in range(3)]
    tol = 1e-12
    for a, (d1, d2) in enumerate([("d1x", "d2x"), ("d1y", "d2y"), ("d1z", "d2z")]):
        got1 = oracle_mod.deriv(f, d1, L, order)
        exp1 = -k_tilde(th[a], h[a]) * s
        assert np.max(np.abs(got1 - exp1)) < tol * max(1.0, abs(k_tilde(th[a], h[a])))
        got2 = oracle_mod.deriv(f, d2, L, order)
        exp2 = beta(th[a]) / h[a] ** 2 * f
        assert np.max(np.abs(got2 - exp2)) < tol * max(1.0, abs(beta(th[a]) / h[a] ** 2))
    for op, (a, b) in (("dxy", (0, 1)), ("dxz", (0, 2)), ("dyz", (1, 2))):
        sym = (beta(th[a] + th[b]) - beta(th[a] - th[b])) / (4 * h[a] * h[b])
        got = oracle_mod.deriv(f, op, L, order)
        assert np.max(np.abs(got - sym * f)) < tol * max(1.0, abs(sym))


def _conv_errors(oracle_mod, op, ns, order=6):
    errs = []
    for n in ns:
        shape = {"d1x": (n, 3, 3), "d2x": (n, 3, 3), "d1y": (3, n, 3), "d2y": (3, n, 3),
                 "d1z": (3, 3, n), "d2z": (3, 3, n), "dxy": (n, n, 3), "dxz": (n, 3, n),
                 "dyz": (3, n, n)}[op]
        X, Y, Z = _grid(shape)
        # a smooth non-trigonometric-polynomial periodic field
        f = np.exp(0.6 * np.sin(X + 0.2) + 0.5 * np.cos(Y - 0.4) + 0.4 * np.sin(Z + 1.0))
        gx = 0.6 * np.cos(X + 0.2)
        gy = -0.5 * np.sin(Y - 0.4)
        gz = 0.4 * np.cos(Z + 1.0)
        exact = {
            "d1x": gx * f, "d1y": gy * f, "d1z": gz * f,
            "d2x": (gx ** 2 - 0.6 * np.sin(X + 0.2)) * f,
            "d2y": (gy ** 2 - 0.5 * np.cos(Y - 0.4)) * f,
            "d2z": (gz ** 2 - 0.4 * np.sin(Z + 1.0)) * f,
            "dxy": gx * gy * f, "dxz": gx * gz * f, "dyz": gy * gz * f,
        }[op]
        errs.append(np.max(np.abs(oracle_mod.deriv(f, op, order=order) - exact)))
    return errs


@pytest.mark.parametrize("op", ["d1x", "d1y", "d1z", "d2x", "d2y", "d2z", "dxy", "dxz", "dyz"])
def test_sixth_order_convergence(oracle_mod, op):
    errs = _conv_errors(oracle_mod, op, [24, 48, 96])
    r1 = errs[0] / errs[1]
    r2 = errs[1] / errs[2]
    # sixth order: 2^6 = 64 per doubling (asymptotically)
    assert 45 < r1 < 90 and 55 < r2 < 75, (errs, r1, r2)


@pytest.mark.parametrize("order", [2, 4, 8])
@pytest.mark.parametrize("op", ["d1x", "d1z", "d2y", "d2z", "dxy", "dyz"])
def test_order_2r_convergence(oracle_mod, op, order):
    errs = _conv_errors(oracle_mod, op, [24, 48, 96], order)
    r1 = errs[0] / errs[1]
    r2 = errs[1] / errs[2]
    rate = 2.0 ** order  # 2^(2r) per doubling, asymptotically
    assert 0.55 * rate < r1 < 1.5 * rate and 0.8 * rate < r2 < 1.2 * rate, (errs, r1, r2)


@pytest.mark.parametrize("order", ORDERS)
def test_periodic_sums_vanish(oracle_mod, order):
    rng = np.random.default_rng(11)
    f = rng.standard_normal((10, 9, 8))
    for op in oracle_mod.OPS:
        d = oracle_mod.deriv(f, op, order=order)
        scale = np.sum(np.abs(d))
        assert abs(np.sum(d)) < 1e-13 * scale


@pytest.mark.parametrize("order", ORDERS)
def test_div_curl_vanishes(oracle_mod, order):
    rng = np.random.default_rng(12)
    A = rng.standard_normal((3, 11, 10, 9))
    d = lambda g, op: oracle_mod.deriv(g, op, order=order)
    Bx = d(A[2], "d1y") - d(A[1], "d1z")
    By = d(A[0], "d1z") - d(A[2], "d1x")
    Bz = d(A[1], "d1x") - d(A[0], "d1y")
    div = d(Bx, "d1x") + d(By, "d1y") + d(Bz, "d1z")
    scale = np.max(np.abs(d(Bx, "d1x")))
    assert np.max(np.abs(div)) < 1e-13 * scale


def test_mixed_is_symmetric_and_diagonal_only(oracle_mod):
    """The mixed operator reads only the planar diagonals (Eq. stencil-fd):
    a field that is zero on both diagonals through a cell yields zero
    there, even if its off-diagonal points are large."""
    n = 16
    f = np.zeros((5, n, n))
    f[2, 1, 2] = 1.0   # off-diagonal neighbour of (x=0, y=0): offsets (2, 1)
    f[2, 3, 1] = -7.0  # offsets (1, 3)
    got = oracle_mod.deriv(f, "dxy")
    assert got[2, 0, 0] == 0.0
    g = np.zeros((5, n, n))
    g[2, 2, 2] = 1.0   # diagonal offset (+2, +2)
    got = oracle_mod.deriv(g, "dxy")
    h = TWO_PI / n
    assert got[2, 0, 0] == pytest.approx((-27 / 180) / (4 * h * h), rel=1e-15)


@pytest.mark.parametrize("order", ORDERS)
def test_stencil_reach_is_the_radius(oracle_mod, order):
    """A unit impulse at axis offset m (and at diagonal offset (m, m)) is
    seen by the order-2r operators exactly when |m| <= r, with the Taylor
    weight of that offset (Eq. stencil-fd: the stencil spans |z| <= r)."""
    r = order // 2
    n = 24
    w1 = _taylor_weights(1, r)
    w2 = _taylor_weights(2, r)
    h = TWO_PI / n
    for m in range(1, 6):
        f = np.zeros((3, 3, n))
        f[1, 1, (5 + m) % n] = 1.0
        got = oracle_mod.deriv(f, "d1x", order=order)[1, 1, 5]
        want = float(w1[m + r]) / h if m <= r else 0.0
        assert got == pytest.approx(want, rel=1e-14, abs=0.0)
        g = np.zeros((3, n, n))
        g[1, (5 + m) % n, (5 + m) % n] = 1.0
        got = oracle_mod.deriv(g, "dxy", order=order)[1, 5, 5]
        want = float(w2[m + r]) / (4 * h * h) if m <= r else 0.0
        assert got == pytest.approx(want, rel=1e-14, abs=0.0)

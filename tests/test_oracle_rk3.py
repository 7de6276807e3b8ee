"""Pins of the oracle's low-storage RK3 update (CPU only).

The paper cites Williamson's third-order 2N scheme (Section 4) without
printing its coefficients.  These checks fix them by what a third-order
2N scheme must satisfy, independently of the printed numbers:
* converted to Butcher form, the coefficients meet all four third-order
  conditions exactly (rational arithmetic);
* one step on y' = lambda y multiplies by exactly 1 + z + z^2/2 + z^3/6;
* on the nonlinear y' = -y^2 the global error falls by 2^3 per halving of dt;
* with alpha_0 = 0 the first substep never reads the old register.
"""
from fractions import Fraction

import numpy as np
import pytest


def _exact_coeffs(oracle_mod):
    a, b = oracle_mod.rk3_coeffs()
    fa = [Fraction(x).limit_denominator(1000) for x in a]
    fb = [Fraction(x).limit_denominator(1000) for x in b]
    for x, fx in zip(list(a) + list(b), fa + fb):
        assert float(fx) == x  # the doubles are the rounded rationals
    return fa, fb


def _butcher_from_2n(alpha, beta):
    """Butcher tableau of the 2N scheme w <- alpha_s w + dt F, y <- y + beta_s w.

    Track each register as a linear combination of the stage slopes k_j:
    w_s = alpha_s w_{s-1} + k_s; y_s = y_{s-1} + beta_s w_s.  Stage s is
    evaluated at y_{s-1}, so a[s][j] = coefficient of k_j in y_{s-1}."""
    S = len(alpha)
    w = [Fraction(0)] * S
    y = [Fraction(0)] * S
    A = [[Fraction(0)] * S for _ in range(S)]
    for s in range(S):
        A[s] = y[:]
        w = [alpha[s] * w[j] + (1 if j == s else 0) for j in range(S)]
        y = [y[j] + beta[s] * w[j] for j in range(S)]
    b = y
    c = [sum(row) for row in A]
    return A, b, c


def test_third_order_conditions_exact(oracle_mod):
    alpha, beta = _exact_coeffs(oracle_mod)
    assert alpha[0] == 0
    A, b, c = _butcher_from_2n(alpha, beta)
    assert sum(b) == 1
    assert sum(bi * ci for bi, ci in zip(b, c)) == Fraction(1, 2)
    assert sum(bi * ci * ci for bi, ci in zip(b, c)) == Fraction(1, 3)
    Ac = [sum(A[i][j] * c[j] for j in range(3)) for i in range(3)]
    assert sum(bi * x for bi, x in zip(b, Ac)) == Fraction(1, 6)
    # explicit: strictly lower triangular
    assert all(A[i][j] == 0 for i in range(3) for j in range(i, 3))


def _rk3_step_scalar(oracle_mod, y0, F, dt):
    f = np.array(y0, dtype=np.float64)
    w = np.full_like(f, np.nan)  # must not be read in substep 0
    for s in range(3):
        r = F(f)
        oracle_mod.rk3_update(s, f, w, np.ascontiguousarray(r), dt)
    return f


@pytest.mark.parametrize("z", [-0.5, -1.2, 0.3, -2.0, 0.05])
def test_amplification_polynomial(oracle_mod, z):
    lam = -3.0
    dt = z / lam
    y = _rk3_step_scalar(oracle_mod, [1.0, 2.5], lambda f: lam * f, dt)
    R = 1 + z + z * z / 2 + z ** 3 / 6
    assert np.allclose(y, [R, 2.5 * R], rtol=1e-14, atol=0)


def test_nonlinear_third_order_convergence(oracle_mod):
    errs = []
    for n in (20, 40, 80, 160):
        dt = 1.0 / n
        y = np.array([1.0])
        for _ in range(n):
            y = _rk3_step_scalar(oracle_mod, y, lambda f: -f * f, dt)
        errs.append(abs(y[0] - 0.5))  # exact y(1) = 1/(1+1)
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(7.0 < r < 9.0 for r in ratios), (errs, ratios)


def test_first_substep_ignores_register(oracle_mod):
    f = np.array([1.0, -2.0, 3.0])
    w = np.array([np.nan, np.inf, -np.inf])
    r = np.array([0.5, 0.25, -1.0])
    oracle_mod.rk3_update(0, f, w, r, 0.1)
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(w))
    assert np.array_equal(w, 0.1 * r)

"""Pins of the oracle's halo mapping, reductions and spot-check entry (CPU only)."""
import math

import numpy as np
import pytest

from paper_2103_01597_amd import inputs


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (4, 4, 4), (7, 6, 9), (32, 5, 3)])
def test_halo_mapping_is_wrap_padding(oracle_mod, shape):
    """Section 3.3's mapping s' = ((s - r) mod n) + r equals periodic
    ('wrap') padding by r on every axis, including n < r."""
    rng = np.random.default_rng(3)
    f = rng.standard_normal((2, *shape[::-1]))
    got = oracle_mod.halo_periodic(f, 3)
    ref = np.pad(f, ((0, 0), (3, 3), (3, 3), (3, 3)), mode="wrap")
    assert np.array_equal(got, ref)


def test_reductions_exact_on_integers(oracle_mod):
    n = 20 * 21 * 22
    x = np.arange(n, dtype=np.float64) - 4000.0
    assert oracle_mod.reduce(x, "sum") == n * (n - 1) / 2 - 4000.0 * n
    k = np.arange(n, dtype=np.float64)
    assert oracle_mod.reduce(x, "sumsq") == float(np.sum((k - 4000) ** 2))  # integers < 2^53
    assert oracle_mod.reduce(x, "maxabs") == max(4000.0, n - 4001.0)
    assert oracle_mod.reduce(x, "min") == -4000.0
    assert oracle_mod.reduce(x, "max") == n - 4001.0
    assert oracle_mod.reduce(np.zeros(17), "sumexp") == 17.0
    y = np.full(10, math.log(2.0))
    assert oracle_mod.reduce(y, "sumexp") == pytest.approx(20.0, rel=1e-15)
    z = np.ones(9)
    z[[1, 4, 7]] = [np.nan, np.inf, -np.inf]
    assert oracle_mod.reduce(z, "nonfinite") == 3.0


def test_fsum_beats_naive_cancellation(oracle_mod):
    x = np.array([1e16, 1.0, -1e16, 1.0])
    assert oracle_mod.reduce(x, "sum") == 2.0


def test_substep_at_equals_full_substep(oracle_mod):
    n = (10, 9, 8)
    p = oracle_mod.Params(*n)
    f0 = inputs.fourier_modes(n, 3, 1e-2, seed=31)
    w0 = inputs.fourier_modes(n, 2, 1e-5, seed=32)
    cells = np.array([0, 5, 77, 9 * 10 * 8 - 1, 123, 456])
    for s in range(3):
        f1, w1 = oracle_mod.substep(s, f0, w0, 1e-3, p)
        fs, ws = oracle_mod.substep_at(s, f0, None if s == 0 else w0, 1e-3, p, cells)
        assert np.array_equal(fs, f1.reshape(8, -1)[:, cells])
        assert np.array_equal(ws, w1.reshape(8, -1)[:, cells])


def test_ulps_definition(oracle_mod):
    m = np.array([1.0, 1.5, 3.0, -0.75])
    eps = np.array([2.0 ** -52, 2.0 ** -52, 2.0 ** -51, 2.0 ** -53])
    c = m + 2 * eps
    assert np.allclose(oracle_mod.ulps(c, m), 2.0)


def test_rel_err_hand_computed(oracle_mod):
    """The parity metric is the infinity-norm relative error max|c - m| /
    max|m| of one field (model m = oracle, candidate c).  Values chosen so
    that every plausible variant gives a different number: the pointwise
    maximum of |c - m| / |m| (0.25), normalising by the candidate (1/7), the
    mean or L2 norms (0.14, 0.145), a signed difference (0.09375), or max(m)
    without the absolute value (1/3)."""
    m = np.array([3.0, -8.0, 1.0, 0.5])
    c = np.array([3.75, -7.0, 1.0, 0.5])
    assert oracle_mod.rel_err(c, m) == 0.125
    assert oracle_mod.rel_err(m, c) == 1.0 / 7.0  # the arguments are not symmetric
    # shape does not matter: the norms run over every element of the field
    assert oracle_mod.rel_err(c.reshape(2, 2), m.reshape(2, 2)) == 0.125
    # identical fields, and an all-zero model (the absolute error is returned)
    assert oracle_mod.rel_err(m, m) == 0.0
    assert oracle_mod.rel_err(np.array([0.0, -2e-3]), np.zeros(2)) == 2e-3
    # one NaN or Inf anywhere in the candidate makes the error non-finite, so
    # no bar of the form err <= tol can pass
    for bad in (np.nan, np.inf):
        cc = c.copy()
        cc[2] = bad
        e = oracle_mod.rel_err(cc, m)
        assert not (e <= 1.0)

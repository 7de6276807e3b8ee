"""Seeded synthetic initial conditions (no arithmetic of the method itself).

Both the GPU path's tests/benchmark and the oracle's tests draw their inputs
from here, so the two sides start from bit-identical states.  Nothing here
evaluates a derivative, a right-hand side or an RK stage.

Fields are float64 arrays of shape (8, nz, ny, nx), x fastest, in the order
of the paper's Table B.1: lnrho, ux, uy, uz, ss, Ax, Ay, Az.

Recipes
-------
* ``fourier_modes``: per field, ``nmodes`` integer wave vectors k drawn
  uniformly from [-kmax, kmax]^3 and kept when 0 < |k| <= kmax (Euclidean),
  then one phase per mode from U[0, 2*pi); value = amp * sum cos(k.x + phi)
  with x = (i h_x, j h_y, k h_z) and wavenumber 2*pi*k/l per axis.  One
  ``numpy.random.default_rng(seed)`` stream serves all 8 fields in order.
* ``uniform01``: i.i.d. U[0, 1) per cell and field -- the random state the
  paper's benchmarks start from (Section 5).
"""
from __future__ import annotations

import math

import numpy as np

NQ = 8
FIELD_NAMES = ("lnrho", "ux", "uy", "uz", "ss", "ax", "ay", "az")


def _draw_modes(rng: np.random.Generator, kmax: int, nmodes: int):
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, size=3)
        k2 = int(k @ k)
        if 0 < k2 <= kmax * kmax:
            ks.append(k)
    phases = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    return np.array(ks), phases


def fourier_mode_fields(shape, kmax: int, amp, seed, nmodes: int = 4,
                        lengths=(2 * math.pi,) * 3, out=None):
    """The fields of ``fourier_modes`` one at a time: yields (q, field) for
    q = 0..7, each field an (nz, ny, nx) float64 array.  By default all
    fields are written into one reused buffer, so that a large state costs
    one field's worth of host memory; ``out`` may name that buffer, or be an
    (8, nz, ny, nx) array that receives field q in out[q]."""
    nx, ny, nz = shape
    amps = np.broadcast_to(np.asarray(amp, dtype=np.float64), (NQ,))
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * (lengths[0] / nx)
    y = np.arange(ny) * (lengths[1] / ny)
    z = np.arange(nz) * (lengths[2] / nz)
    single = np.empty((nz, ny, nx), dtype=np.float64) if out is None else out
    for q in range(NQ):
        buf = single[q] if single.ndim == 4 else single
        ks, phases = _draw_modes(rng, kmax, nmodes)
        # cos(a_x x + a_y y + a_z z + phi) = cos(a_z z + phi) C(x, y) - sin(a_z z + phi) S(x, y)
        # with C, S the cosine/sine of a_x x + a_y y: one (nz, 2m) x (2m, ny*nx) product.
        zfac = np.empty((nz, 2 * nmodes))
        xyfac = np.empty((2 * nmodes, ny * nx))
        for m, ((kx, ky, kz), ph) in enumerate(zip(ks, phases)):
            ax = 2 * math.pi * kx / lengths[0]
            ay = 2 * math.pi * ky / lengths[1]
            az = 2 * math.pi * kz / lengths[2]
            cx, sx = np.cos(ax * x), np.sin(ax * x)
            cy, sy = np.cos(ay * y), np.sin(ay * y)
            xyfac[2 * m] = (cy[:, None] * cx[None, :] - sy[:, None] * sx[None, :]).ravel()
            xyfac[2 * m + 1] = (sy[:, None] * cx[None, :] + cy[:, None] * sx[None, :]).ravel()
            zfac[:, 2 * m] = amps[q] * np.cos(az * z + ph)
            zfac[:, 2 * m + 1] = -amps[q] * np.sin(az * z + ph)
        np.matmul(zfac, xyfac, out=buf.reshape(nz, ny * nx))
        yield q, buf


def fourier_modes(shape, kmax: int, amp, seed, nmodes: int = 4,
                  lengths=(2 * math.pi,) * 3, dtype=np.float64) -> np.ndarray:
    """Sum-of-Fourier-modes state. ``shape`` = (nx, ny, nz); ``amp`` is a
    scalar or 8 per-field amplitudes (a zero amplitude still draws its modes
    so the other fields do not depend on it)."""
    nx, ny, nz = shape
    out = np.empty((NQ, nz, ny, nx), dtype=np.float64)
    for _ in fourier_mode_fields(shape, kmax, amp, seed, nmodes, lengths, out=out):
        pass
    return out.astype(dtype, copy=False)


def uniform01(shape, seed, dtype=np.float64) -> np.ndarray:
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    return rng.random((NQ, nz, ny, nx)).astype(dtype, copy=False)


# Named workloads: grid, initial condition and integration settings.
# Physics constants shared by all: cs0 = 1, gamma = 5/3, nu = eta = 5e-3,
# K = rho0 cp chi = 5e-3 (chi = 5e-3), cp = 1, mu0 = 1, lnrho0 = 0.
WORKLOADS = {
    "oracle32": dict(shape=(32, 32, 32), kmax=3, amp=1e-2, seed=1, dt=1e-3, steps=1),
    "sub256": dict(shape=(256, 256, 256), kmax=8, amp=1e-2, seed=2, dt=1e-3, steps=100),
    "prec512": dict(shape=(512, 512, 512), kmax=8, amp=1e-2, seed=3, dt=1e-3, steps=100),
    # the paper's own benchmark state (Section 5): i.i.d. U[0, 1) fields, dt = 2^-23
    "w0_512": dict(shape=(512, 512, 512), init="uniform01", seed=0, dt=2.0 ** -23, steps=100),
    "large1024x512x512": dict(shape=(1024, 512, 512), kmax=16,
                              amp=(0.0, 0.1, 0.1, 0.1, 0.0, 1e-3, 1e-3, 1e-3),
                              seed=4, dt=1e-3, steps=50,
                              lengths=(4 * math.pi, 2 * math.pi, 2 * math.pi)),
}


def workload_state(name: str, dtype=np.float64, shape=None) -> np.ndarray:
    """Initial state of a named workload (optionally on another grid shape)."""
    w = WORKLOADS[name]
    if w.get("init") == "uniform01":
        return uniform01(shape or w["shape"], w["seed"], dtype=dtype)
    return fourier_modes(shape or w["shape"], w["kmax"], w["amp"], w["seed"],
                         lengths=w.get("lengths", (2 * math.pi,) * 3), dtype=dtype)


def uniform01_fields(shape, seed):
    """The fields of ``uniform01`` one at a time, (q, (nz, ny, nx) array);
    bit-identical to ``uniform01`` (the same generator stream, in order)."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    for q in range(NQ):
        yield q, rng.random((nz, ny, nx))


def workload_fields(name: str, shape=None):
    """``workload_state`` one field at a time (see ``fourier_mode_fields``)."""
    w = WORKLOADS[name]
    if w.get("init") == "uniform01":
        return uniform01_fields(shape or w["shape"], w["seed"])
    return fourier_mode_fields(shape or w["shape"], w["kmax"], w["amp"], w["seed"],
                               lengths=w.get("lengths", (2 * math.pi,) * 3))

"""CPU oracle for the fused MHD RK3 substep (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and this package never
imports the product.

Contents
--------
* :func:`rhs`, :func:`substep`, :func:`step`, :func:`deriv`: ctypes wrappers
  of ``mhd_oracle.c`` (plain FP64 C, modulo indexing, no halo), which follows
  Section 4 (Eq. stencil-fd), Appendix B (Eqs. B.1-B.4) and the Williamson
  2N RK3 the paper cites in Section 4.
* :func:`halo_periodic`: the periodic halo mapping of Section 3.3,
  s' = ((s - r) mod n) + r, written out with index arithmetic.
* :func:`reduce`: the reductions by their definitions (``math.fsum`` etc.).
* :func:`ulps`: the paper's ulp error measure (Section 5).

Arrays are NumPy float64 of shape (8, nz, ny, nx), x fastest, in the field
order of Table B.1: lnrho, ux, uy, uz, ss, Ax, Ay, Az.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libmhd_oracle.so")
_lib = None

NQ = 8
FIELD_NAMES = ("lnrho", "ux", "uy", "uz", "ss", "ax", "ay", "az")
R = 3  # default stencil radius (Section 2, Eq. 1; sixth order: k = 2r)
ORDERS = (2, 4, 6, 8)  # the stencil orders of Section 4 (radius r = order / 2)

OPS = {"d1x": 0, "d1y": 1, "d1z": 2, "d2x": 3, "d2y": 4, "d2z": 5,
       "dxy": 6, "dxz": 7, "dyz": 8}


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("radius", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("cs0", ctypes.c_double), ("gamma", ctypes.c_double), ("cp", ctypes.c_double),
                ("lnrho0", ctypes.c_double), ("mu0", ctypes.c_double), ("nu", ctypes.c_double),
                ("zeta", ctypes.c_double), ("eta", ctypes.c_double), ("K", ctypes.c_double),
                ("bext", ctypes.c_double * 3), ("heat", ctypes.c_double), ("cool", ctypes.c_double)]


@dataclass
class Params:
    """Grid and physics constants (the oracle's own copy of the defaults)."""
    nx: int
    ny: int
    nz: int
    lx: float = 2 * math.pi
    ly: float = 2 * math.pi
    lz: float = 2 * math.pi
    cs0: float = 1.0
    gamma: float = 5.0 / 3.0
    cp: float = 1.0
    lnrho0: float = 0.0
    mu0: float = 1.0
    nu: float = 5e-3
    zeta: float = 0.0
    eta: float = 5e-3
    K: float = 5e-3
    bext: tuple = field(default=(0.0, 0.0, 0.0))
    order: int = 6  # stencil order k = 2r (Section 4)
    heat: float = 0.0  # explicit heating H of Eq. B.3 (uniform)
    cool: float = 0.0  # explicit cooling C of Eq. B.3 (uniform)

    def _c(self) -> _Params:
        p = _Params()
        p.radius = _radius(self.order)
        for name in ("nx", "ny", "nz", "lx", "ly", "lz", "cs0", "gamma", "cp", "lnrho0",
                     "mu0", "nu", "zeta", "eta", "K", "heat", "cool"):
            setattr(p, name, getattr(self, name))
        p.bext = (ctypes.c_double * 3)(*[float(b) for b in self.bext])
        return p


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Params)
    lib.oracle_deriv.argtypes = ([ctypes.c_int32] * 3 + [ctypes.c_double] * 3 +
                                 [ctypes.c_int32, dp, ctypes.c_int32, dp])
    lib.oracle_weights.argtypes = [ctypes.c_int32, dp, dp]
    lib.oracle_rk3_coeffs.argtypes = [dp, dp]
    lib.oracle_rhs.argtypes = [pp, dp, dp]
    lib.oracle_rk3_update.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, dp, dp, ctypes.c_double]
    lib.oracle_substep.argtypes = [pp, ctypes.c_int32, dp, dp, ctypes.c_double, dp]
    lib.oracle_step.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_int32]
    lib.oracle_substep_at.argtypes = [pp, ctypes.c_int32, dp, dp, ctypes.c_double, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64), dp, dp]
    for fn in ("oracle_deriv", "oracle_weights", "oracle_rhs", "oracle_rk3_update", "oracle_substep", "oracle_step",
               "oracle_substep_at"):
        getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _fields(f: np.ndarray, p: Params) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.shape != (NQ, p.nz, p.ny, p.nx):
        raise ValueError(f"expected shape {(NQ, p.nz, p.ny, p.nx)}, got {f.shape}")
    return f


def _radius(order: int) -> int:
    if order not in ORDERS:
        raise ValueError(f"stencil order must be one of {ORDERS}, got {order}")
    return order // 2


def weights(order: int = 6):
    """(a1, a2): the first/second-derivative weights for offsets -r..r."""
    r = _radius(order)
    a1 = np.zeros(2 * r + 1)
    a2 = np.zeros(2 * r + 1)
    if _load().oracle_weights(r, _ptr(a1), _ptr(a2)) != 0:
        raise ValueError("oracle_weights failed")
    return a1, a2


def rk3_coeffs():
    a = np.zeros(3)
    b = np.zeros(3)
    _load().oracle_rk3_coeffs(_ptr(a), _ptr(b))
    return a, b


def deriv(f: np.ndarray, op: str, lengths=(2 * math.pi,) * 3, order: int = 6) -> np.ndarray:
    """One derivative operator of the given stencil order on one periodic
    field of shape (nz, ny, nx)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    rc = _load().oracle_deriv(nx, ny, nz, *[float(x) for x in lengths], _radius(order), _ptr(f),
                              OPS[op], _ptr(out))
    if rc != 0:
        raise ValueError("oracle_deriv failed")
    return out


def rhs(f: np.ndarray, p: Params) -> np.ndarray:
    f = _fields(f, p)
    out = np.empty_like(f)
    cp = p._c()
    if _load().oracle_rhs(ctypes.byref(cp), _ptr(f), _ptr(out)) != 0:
        raise ValueError("oracle_rhs failed")
    return out


def rk3_update(s: int, f: np.ndarray, w: np.ndarray, r: np.ndarray, dt: float) -> None:
    """In-place 2N update of flat float64 arrays f, w with right-hand side r."""
    for a in (f, w, r):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    if _load().oracle_rk3_update(f.size, s, _ptr(f), _ptr(w), _ptr(r), dt) != 0:
        raise ValueError("oracle_rk3_update failed")


def substep(s: int, f: np.ndarray, w: np.ndarray, dt: float, p: Params):
    """Return (f', w') after RK3 substep s (inputs are not modified)."""
    f = _fields(f, p).copy()
    w = np.ascontiguousarray(w, dtype=np.float64).copy()
    scratch = np.empty_like(f)
    cp = p._c()
    if _load().oracle_substep(ctypes.byref(cp), s, _ptr(f), _ptr(w), dt, _ptr(scratch)) != 0:
        raise ValueError("oracle_substep failed")
    return f, w


def substep_at(s: int, f: np.ndarray, w, dt: float, p: Params, cells: np.ndarray):
    """Substep s at selected flat interior cells only: returns (f', w') of
    shape (8, len(cells)).  ``w`` may be None for s = 0."""
    f = _fields(f, p)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    nc = cells.size
    out_f = np.empty((NQ, nc))
    out_w = np.empty((NQ, nc))
    wp = None
    if w is not None:
        w = _fields(w, p)
        wp = _ptr(w)
    cp = p._c()
    rc = _load().oracle_substep_at(ctypes.byref(cp), s, _ptr(f), wp, dt, nc,
                                   cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   _ptr(out_f), _ptr(out_w))
    if rc != 0:
        raise ValueError("oracle_substep_at failed")
    return out_f, out_w


def step(f: np.ndarray, dt: float, p: Params, nsteps: int = 1) -> np.ndarray:
    """Return the state after nsteps full RK3 steps (input not modified)."""
    f = _fields(f, p).copy()
    w = np.zeros_like(f)
    cp = p._c()
    if _load().oracle_step(ctypes.byref(cp), _ptr(f), _ptr(w), dt, nsteps) != 0:
        raise ValueError("oracle_step failed")
    return f


# ------------------------------------------------------------------ halo
def halo_periodic(f: np.ndarray, r: int = R) -> np.ndarray:
    """Periodic halo fill by the mapping of Section 3.3.

    ``f`` holds the computational domain, shape (..., nz, ny, nx).  The
    result has shape (..., nz+2r, ny+2r, nx+2r); grid index s along an axis
    of n interior cells holds interior cell ((s - r) mod n) + r, i.e. the
    interior value at unpadded index (s - r) mod n.
    """
    f = np.asarray(f)
    *lead, nz, ny, nx = f.shape
    iz = np.array([(s - r) % nz for s in range(nz + 2 * r)])
    iy = np.array([(s - r) % ny for s in range(ny + 2 * r)])
    ix = np.array([(s - r) % nx for s in range(nx + 2 * r)])
    return f[..., iz[:, None, None], iy[None, :, None], ix[None, None, :]]


# ------------------------------------------------------------- reductions
REDUCE_OPS = ("sum", "sumsq", "maxabs", "min", "max", "sumexp", "nonfinite")


def reduce(field_values: np.ndarray, op: str) -> float:
    """Reduction of one field's interior by its definition."""
    x = np.asarray(field_values, dtype=np.float64).ravel()
    if op == "sum":
        return math.fsum(x.tolist())
    if op == "sumsq":
        return math.fsum((x * x).tolist())
    if op == "maxabs":
        return float(np.max(np.abs(x)))
    if op == "min":
        return float(np.min(x))
    if op == "max":
        return float(np.max(x))
    if op == "sumexp":
        return math.fsum(np.exp(x).tolist())
    if op == "nonfinite":
        return float(np.count_nonzero(~np.isfinite(x)))
    raise ValueError(op)


# -------------------------------------------------------------- metrics
def ulps(candidate: np.ndarray, model: np.ndarray, p: int = 53) -> np.ndarray:
    """Absolute error in units of the model value's last place (Section 5):
    eps = 2**(floor(log2|m|) - p + 1); undefined (NaN) where m == 0."""
    m = np.asarray(model, dtype=np.float64)
    c = np.asarray(candidate, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        e = np.floor(np.log2(np.abs(m)))
        eps = np.exp2(e - p + 1)
        out = np.abs(m - c) / eps
    out[m == 0] = np.nan
    return out


def rel_err(candidate: np.ndarray, model: np.ndarray) -> float:
    """Infinity-norm relative error max|c - m| / max|m| of one field."""
    m = np.asarray(model, dtype=np.float64)
    c = np.asarray(candidate, dtype=np.float64)
    den = np.max(np.abs(m))
    num = np.max(np.abs(c - m))
    return float(num / den) if den > 0 else float(num)

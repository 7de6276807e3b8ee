"""Oracle values at sampled cells of a grid too large for the oracle.

A cell's state after k substeps depends only on the initial state within
rk cells of it (each substep reads a stencil of radius r = order / 2, 3 at
sixth order).  So for every sampled cell the oracle runs the k substeps on
a small periodic block (side at least 2rk + 1, same grid spacing) cut, with
periodic wrap, from the full initial state around that cell; the value
there is then exactly the full-grid oracle's (the block's own periodic wrap
only corrupts cells within rj of its faces after j substeps).  The input is the seeded initial state; nothing comes
from the GPU path.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

import oracle
from paper_2103_01597_amd import inputs


def _block_side(length, n, r):
    """Smallest block side m >= 2r + 1 and a length l_b with l_b / m ==
    length / n exactly in float64, so that the block has the full grid's
    spacing to the last bit (not every side reaches a given spacing)."""
    h = length / n
    for m in range(2 * r + 1, 4 * r + 8):
        lb = h * m
        for cand in (lb, np.nextafter(lb, np.inf), np.nextafter(lb, -np.inf)):
            if cand / m == h:
                return m, float(cand)
    raise ValueError("no block side reproduces the grid spacing")


def block_reference(f0, cells, p: "oracle.Params", dt: float, nsub: int):
    """f0: (8, nz, ny, nx) initial state; cells: (k, j, i) index arrays.
    Returns (fs, ws), each (nsub, 8, ncells): the oracle's state and 2N
    register at every sampled cell after substeps 1..nsub of consecutive
    RK3 steps (substep index cycling 0, 1, 2)."""
    k, j, i = (np.asarray(a, dtype=np.int64) for a in cells)
    nz, ny, nx = f0.shape[1:]
    r = (p.order // 2) * nsub
    (mx, lx), (my, ly), (mz, lz) = (_block_side(p.lx, nx, r), _block_side(p.ly, ny, r),
                                    _block_side(p.lz, nz, r))
    if mx > nx or my > ny or mz > nz:
        raise ValueError("grid smaller than the dependence block")
    pb = dataclasses.replace(p, nx=mx, ny=my, nz=mz, lx=lx, ly=ly, lz=lz)
    # the sampled cell sits r cells from the low faces of its block, at
    # least r from the high faces
    fs = np.empty((nsub, 8, k.size))
    ws = np.empty((nsub, 8, k.size))
    for c in range(k.size):
        iz = (k[c] - r + np.arange(mz)) % nz
        iy = (j[c] - r + np.arange(my)) % ny
        ix = (i[c] - r + np.arange(mx)) % nx
        blk = np.ascontiguousarray(f0[np.ix_(np.arange(8), iz, iy, ix)], dtype=np.float64)
        w = np.zeros_like(blk)
        for t in range(nsub):
            blk, w = oracle.substep(t % 3, blk, w, dt, pb)
            fs[t, :, c] = blk[:, r, r, r]
            ws[t, :, c] = w[:, r, r, r]
    return fs, ws


def sample_cells(n, ncells, seed):
    """ncells seeded random interior cells of an (nx, ny, nz) grid plus its
    first and last cells and the ends of its first row and plane, as
    (k, j, i) index arrays."""
    rng = np.random.default_rng(seed)
    total = n[0] * n[1] * n[2]
    cells = np.unique(np.concatenate([rng.integers(0, total, ncells),
                                      [0, total - 1, n[0] - 1, n[0] * n[1] - 1]]))
    k, rem = np.divmod(cells, n[0] * n[1])
    j, i = np.divmod(rem, n[0])
    return k, j, i


_CACHE = {}


def workload_reference(wl_name, ncells=400, seed=0, fp32_state=False, order=6):
    """(params, initial state, cells, fs, ws, per-field max |f0|) for one
    RK3 step of a named workload, fs/ws from block_reference.  With
    fp32_state the initial state is first rounded to FP32 (the state an
    FP32-storage run starts from), so that a comparison measures the
    arithmetic and storage of the run, not the rounding of its input; order
    is the stencil order of the oracle (and of the run compared).  The
    most recent workload is cached (the state of a large one is
    gigabytes)."""
    key = (wl_name, ncells, seed, fp32_state, order)
    if key not in _CACHE:
        _CACHE.clear()
        wl = inputs.WORKLOADS[wl_name]
        n = wl["shape"]
        lengths = wl.get("lengths", (2 * math.pi,) * 3)
        p = oracle.Params(*n, lx=lengths[0], ly=lengths[1], lz=lengths[2], order=order)
        f0 = inputs.workload_state(wl_name)
        if fp32_state:
            f0 = f0.astype(np.float32).astype(np.float64)
        cells = sample_cells(n, ncells, seed)
        fs, ws = block_reference(f0, cells, p, wl["dt"], 3)
        scale = np.abs(f0).reshape(8, -1).max(axis=1)
        _CACHE[key] = (p, f0, cells, fs, ws, scale)
    return _CACHE[key]

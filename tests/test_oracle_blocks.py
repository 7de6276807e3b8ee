"""The dependence-block evaluation used by the full-size sampled parity
tests reproduces the full-grid oracle exactly at the sampled cells."""
import numpy as np

import oracle
from oracle_blocks import block_reference, sample_cells
from paper_2103_01597_amd import inputs


def test_blocks_equal_full_grid_oracle():
    n = (40, 36, 32)
    p = oracle.Params(*n, lx=5.0, ly=4.0, lz=3.5, zeta=2e-3, bext=(0.1, -0.2, 0.05))
    f0 = inputs.fourier_modes(n, 3, 0.05, seed=7, lengths=(5.0, 4.0, 3.5))
    cells = sample_cells(n, 25, seed=3)
    dt = 1e-3
    fs, ws = block_reference(f0, cells, p, dt, 3)
    f, w = f0.copy(), np.zeros_like(f0)
    for s in range(3):
        f, w = oracle.substep(s, f, w, dt, p)
        assert np.array_equal(fs[s], f[(slice(None),) + cells])
        assert np.array_equal(ws[s], w[(slice(None),) + cells])


def test_blocks_equal_full_grid_oracle_orders_2_and_8():
    """The same at stencil orders 2 and 8 (blocks of radius 3 and 12 cells
    around each sampled cell after three substeps)."""
    for order in (2, 8):
        n = (28, 26, 27) if order == 8 else (16, 14, 12)
        p = oracle.Params(*n, lx=3.0, ly=2.5, lz=2.0, order=order, bext=(0.1, 0.0, -0.1))
        f0 = inputs.fourier_modes(n, 3, 0.05, seed=11, lengths=(3.0, 2.5, 2.0))
        cells = sample_cells(n, 6, seed=4)
        dt = 1e-3
        fs, ws = block_reference(f0, cells, p, dt, 3)
        f, w = f0.copy(), np.zeros_like(f0)
        for s in range(3):
            f, w = oracle.substep(s, f, w, dt, p)
            assert np.array_equal(fs[s], f[(slice(None),) + cells])
            assert np.array_equal(ws[s], w[(slice(None),) + cells])

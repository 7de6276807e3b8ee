"""GPU tests of the stencil orders 2, 4, 6 and 8 (Section 4: central
differences of order k = 2r on the stencil set of Eq. stencil-fd), through
the C ABI, against the FP64 oracle at the same order.

Bars: the halo fill of width r is bit-identical to the periodic mapping
s' = ((s - r) mod n) + r; FP64 full steps match the oracle to 1e-11 per
field (infinity-norm relative error); one FP32C step from the same
FP32-rounded start to 1.5e-7 (observed 4.6e-8 at orders 2, 4 and 8 for every
kernel, as at sixth order: half an ulp of storage rounding plus the FP32
first derivatives), one plain FP32 step (no compensation, FP32
second-derivative sums) to 3.5e-7 (observed 1.1e-7); the segmented step
is bit-identical to the monolithic one at every order; init accepts exactly
the kernel/order/precision combinations that are built.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2103_01597_amd import inputs

pytestmark = pytest.mark.gpu
TOL_F64 = 1e-11
TOL_F32C = 1.5e-7
TOL_F32 = 3.5e-7


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mhd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2103_01597_amd import mhd as m
    m.lib()
    return m


def _phys_kw(p):
    return dict(lengths=(p.lx, p.ly, p.lz), cs0=p.cs0, gamma=p.gamma, cp=p.cp, lnrho0=p.lnrho0,
                mu0=p.mu0, nu=p.nu, zeta=p.zeta, eta=p.eta, K=p.K, bext=p.bext)


def _params(shape, order):
    return oracle.Params(*shape, lx=2 * math.pi * shape[0] / 32, ly=2 * math.pi * shape[1] / 32,
                         lz=2 * math.pi * shape[2] / 32, nu=0.02, eta=0.01, K=0.01, zeta=0.003,
                         bext=(0.02, -0.01, 0.03), order=order)


def _run(mhd, f0, p, dt, nsteps, prec, kernel):
    import torch
    S = mhd.Solver(p.nx, p.ny, p.nz, prec, kernel, order=p.order, **_phys_kw(p))
    a = S.upload(f0)
    b = S.empty()
    b.fill_(float("nan"))
    w = S.empty()
    w.fill_(float("nan"))
    comp = S.zeros() if prec == "f32c" else None
    cur = S.step([a, b], 0, w, comp, dt, nsteps)
    torch.cuda.synchronize()
    out = S.download([a, b][cur])
    used = S.kernel
    S.close()
    return out, used


@pytest.mark.parametrize("order", [2, 4, 8])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(20, 17, 11), (1, 2, 5), (3, 9, 4), (40, 6, 9)])
def test_halo_fill_width_r(mhd, shape, prec, order):
    import torch
    say(f"halo {shape} {prec} order {order}")
    r = order // 2
    S = mhd.Solver(*shape, prec, order=order)
    assert S.r == r and S.layout.mx == shape[0] + 2 * r
    f0 = inputs.fourier_modes(shape, 3, 0.5, seed=31)
    buf = S.upload(f0, fill_halo=False)
    S.grid_view(buf).fill_(float("nan"))
    S.interior_view(buf).copy_(torch.from_numpy(f0).to(S.torch_dtype))
    S.halo_periodic(buf)
    torch.cuda.synchronize()
    got = S.grid_view(buf).double().cpu().numpy()
    src = f0 if prec == "f64" else f0.astype(np.float32).astype(np.float64)
    assert np.array_equal(got, oracle.halo_periodic(src, r))
    S.close()


CASES = [(2, "tiled"), (2, "direct"), (2, "split"), (4, "tiled"), (4, "direct"), (4, "split"),
         (6, "tiled"), (8, "tiled"), (8, "direct"), (8, "split")]


@pytest.mark.parametrize("order,kernel", CASES)
@pytest.mark.parametrize("shape", [(32, 32, 32), (37, 29, 31), (20, 12, 70), (5, 7, 6)])
def test_f64_step_against_oracle(mhd, shape, order, kernel):
    say(f"f64 order {order} {kernel} {shape}")
    p = _params(shape, order)
    f0 = inputs.fourier_modes(shape, 3, 0.05, seed=41, lengths=(p.lx, p.ly, p.lz))
    got, used = _run(mhd, f0, p, 2e-3, 2, "f64", kernel)
    assert used == kernel
    ref = oracle.step(f0, 2e-3, p, 2)
    e = [oracle.rel_err(got[q], ref[q]) for q in range(8)]
    say("  rel err:", ["%.2e" % x for x in e])
    assert max(e) <= TOL_F64


@pytest.mark.parametrize("order,kernel", [(2, "tiled"), (4, "tiled"), (8, "tiled"), (8, "direct"),
                                          (2, "split"), (4, "split"), (8, "split")])
@pytest.mark.parametrize("shape", [(32, 32, 32), (37, 29, 31), (20, 12, 70)])
def test_f32c_step_against_oracle(mhd, shape, order, kernel):
    say(f"f32c order {order} {kernel} {shape}")
    p = _params(shape, order)
    f0 = inputs.fourier_modes(shape, 3, 0.05, seed=42, lengths=(p.lx, p.ly, p.lz))
    f0 = f0.astype(np.float32).astype(np.float64)  # both sides start from the same state
    got, used = _run(mhd, f0, p, 2e-3, 1, "f32c", kernel)
    assert used == kernel
    ref = oracle.step(f0, 2e-3, p, 1)
    e = [oracle.rel_err(got[q], ref[q]) for q in range(8)]
    say("  rel err:", ["%.2e" % x for x in e])
    assert max(e) <= TOL_F32C


@pytest.mark.parametrize("order,kernel", [(2, "tiled"), (4, "tiled"), (6, "tiled"), (8, "tiled"),
                                          (8, "direct"), (2, "split"), (4, "split"), (8, "split")])
@pytest.mark.parametrize("shape", [(32, 32, 32), (37, 29, 31), (20, 12, 70)])
def test_f32_step_against_oracle(mhd, shape, order, kernel):
    """Plain FP32 (no compensation, FP32 second-derivative sums) at every
    order, one step from the same FP32-rounded state as the oracle."""
    say(f"f32 order {order} {kernel} {shape}")
    p = _params(shape, order)
    f0 = inputs.fourier_modes(shape, 3, 0.05, seed=43, lengths=(p.lx, p.ly, p.lz))
    f0 = f0.astype(np.float32).astype(np.float64)
    got, used = _run(mhd, f0, p, 2e-3, 1, "f32", kernel)
    assert used == kernel
    ref = oracle.step(f0, 2e-3, p, 1)
    e = [oracle.rel_err(got[q], ref[q]) for q in range(8)]
    say("  rel err:", ["%.2e" % x for x in e])
    assert max(e) <= TOL_F32


@pytest.mark.parametrize("order", [2, 4, 8])
def test_order_study_size_sampled(mhd, order):
    """The order study's configuration (256^3, the sub256 state, FP64, the
    kernel AUTO picks, mhd_step): one RK3 step compared at 100 sampled cells
    with the oracle at the same order run on dependence blocks of the
    initial state (radius 3r around each cell after the three substeps)."""
    import torch
    from oracle_blocks import workload_reference
    wl = inputs.WORKLOADS["sub256"]
    n = wl["shape"]
    p, f0, cells, fs, ws, scale = workload_reference("sub256", 100, 1, order=order)
    S = mhd.Solver(*n, "f64", None, order=order, **_phys_kw(p))
    say(f"sampled 256^3 order {order}: kernel {S.kernel}")
    bufs = [S.upload(f0), S.empty()]
    w = S.zeros()
    cur = S.step(bufs, 0, w, None, wl["dt"], 1)
    torch.cuda.synchronize()
    idx = (slice(None),) + tuple(torch.as_tensor(a) for a in cells)
    gf = S.interior_view(bufs[cur])[idx].cpu().numpy()
    gw = S.interior_view(w)[idx].cpu().numpy()
    S.close()
    ef = [np.max(np.abs(gf[q] - fs[2, q])) / scale[q] for q in range(8)]
    ew = [np.max(np.abs(gw[q] - ws[2, q])) / max(np.max(np.abs(ws[2, q])), 1e-300)
          for q in range(8)]
    say("  f rel err:", ["%.2e" % e for e in ef])
    say("  w rel err:", ["%.2e" % e for e in ew])
    assert max(ef) <= TOL_F64 and max(ew) <= TOL_F64


def test_orders_differ(mhd):
    """The order really reaches the kernels: at a coarse resolution the
    results of different orders differ far beyond rounding."""
    shape = (16, 16, 16)
    outs = []
    for order in (2, 4, 6, 8):
        p = _params(shape, order)
        f0 = inputs.fourier_modes(shape, 5, 0.05, seed=43, lengths=(p.lx, p.ly, p.lz))
        outs.append(_run(mhd, f0, p, 2e-3, 1, "f64", None)[0])
    for i in range(4):
        for j in range(i + 1, 4):
            assert oracle.rel_err(outs[i][1], outs[j][1]) > 1e-6


def test_kernel_availability(mhd):
    auto = {("f64", 2): "split", ("f64", 4): "split", ("f64", 6): "split", ("f64", 8): "split",
            ("f32c", 2): "tiled", ("f32c", 6): "tiled", ("f32c", 8): "split", ("f32", 6): "tiled",
            ("f32", 8): "split"}
    for (prec, order), kernel in auto.items():
        S = mhd.Solver(16, 16, 16, prec, order=order)
        assert S.kernel == kernel and S.r == order // 2
        S.close()
    for prec, order in [("f64", 2), ("f64", 4), ("f64", 8), ("f32c", 8), ("f32", 2)]:
        S = mhd.Solver(16, 16, 16, prec, "split", order=order)
        assert S.kernel == "split" and S.r == order // 2
        S.close()
    with pytest.raises(mhd.MhdError):
        mhd.Solver(16, 16, 16, "f64", order=3)


@pytest.mark.parametrize("order", [2, 4, 8])
@pytest.mark.parametrize("prec", ["f64", "f32c"])
@pytest.mark.parametrize("kernel", [None, "split"])
def test_segmented_step_equals_step(mhd, order, prec, kernel):
    import torch
    n = (72, 40, 48)
    say(f"segmented order {order} {prec} {kernel}")
    S = mhd.Solver(*n, prec, kernel, order=order)
    f0 = inputs.fourier_modes(n, 3, 0.05, seed=44)
    comm = torch.cuda.Stream()
    res = []
    for segmented in (False, True):
        f = [S.upload(f0), S.empty()]
        w = S.zeros()
        comp = S.zeros() if prec == "f32c" else None
        if segmented:
            cur = S.step_segmented(f, 0, w, comp, 1e-3, 2, comm_stream=comm)
        else:
            cur = S.step(f, 0, w, comp, 1e-3, 2)
        torch.cuda.synchronize()
        res.append((cur, S.interior_view(f[cur]).cpu().numpy()))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
    S.close()

"""GPU parity at the full size of every benchmarked workload, and the error
of the FP32-storage variants at 512^3 against the GPU FP64 path.

* The large domain (1024 x 512 x 512 on a 4pi x 2pi x 2pi box, the only
  workload with unequal sides and lengths) and the paper's own benchmark
  state (i.i.d. U[0, 1) per cell and field, dt = 2^-23, Section 5) run one
  full RK3 step through mhd_step with the kernel AUTO picks, i.e. the
  launch configuration the benchmark times.  The outputs are compared at
  about 400 sampled cells with the oracle run on dependence blocks of the
  seeded initial state (a cell after one step depends only on the state
  within 3 x 3 cells of it).  FP64: infinity-norm relative error per field
  over the sampled cells <= 1e-11 (normalised by the largest sampled oracle
  value: ln rho and s of the large domain start at zero), with the paper's
  ulp measure printed beside it.  FP32C: the oracle starts from the
  same FP32-rounded state and the bar is the FP32C one.
* FP32C and plain FP32 against FP64 on the GPU at 512^3 after 1 and 100
  steps, every interior cell, all three runs from the same FP32-rounded
  state (the FP64 path itself is held to the oracle by the sampled 512^3
  parity tests).
"""
import sys

import numpy as np
import pytest

import oracle
from oracle_blocks import workload_reference
from paper_2103_01597_amd import inputs

pytestmark = pytest.mark.gpu
TOL_F64 = 1e-11
# FP32 bars, about three times the largest error observed on MI355X.
# FP32C after one step against the FP64 oracle, both from the same FP32
# state: the result is rounded to FP32 once (half an ulp, 3e-8 of the field's
# largest value), plus the FP32 first derivatives.  Fields that start at
# zero (ln rho and s of the large domain) carry, relative to their own small
# size after one step, the relative error of their right-hand side, whose
# FP32 first derivatives see the rounding of the O(0.1) velocity: observed
# 2.8e-7 (ln rho) and 2.3e-6 (s).
TOL_F32C_1 = 1.5e-7
TOL_F32C_1_FROM_ZERO = 7e-6
TOL_F32C_W0 = 2e-7          # observed 6.2e-8
# 512^3 against the GPU FP64 path: the Lorentz force takes second
# differences of A's FP32 rounding (amplified by 1/h^2), which puts about 4
# ulps into u per step: observed 3.9e-7 after 1 step, 4.2e-7 after 100 steps
# (plain FP32: 8.9e-7 and 8.0e-6).
TOL_F32C_512_1 = 1.2e-6
TOL_F32C_512_100 = 1.3e-6
TOL_F32_512_100 = 2.4e-5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def mhd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2103_01597_amd import mhd as m
    m.lib()
    return m


def _sampled_full_step(mhd, wl_name, prec, ncells=400):
    """One RK3 step of a named workload at full size via mhd_step (AUTO
    kernel); returns per-field (rel err of f, rel err of w, max ulps of f)."""
    import torch
    wl = inputs.WORKLOADS[wl_name]
    n = wl["shape"]
    p, f0, cells, fs, ws, scale = workload_reference(wl_name, ncells, fp32_state=(prec != "f64"))
    S = mhd.Solver(*n, prec, lengths=(p.lx, p.ly, p.lz))
    say(f"{wl_name} {n} {prec}: kernel {S.layout.kernel}, "
        f"{3 * S.layout.total_elems * S.layout.elem_size / 1e9:.1f} GB of f/w buffers")
    bufs = [S.upload(f0), S.empty()]
    w = S.empty()
    comp = S.zeros() if prec == "f32c" else None
    cur = S.step(bufs, 0, w, comp, wl["dt"], 1)
    torch.cuda.synchronize()
    idx = (slice(None),) + tuple(torch.as_tensor(a) for a in cells)
    gf = S.interior_view(bufs[cur])[idx].cpu().double().numpy()
    gw = S.interior_view(w)[idx].cpu().double().numpy()
    S.close()
    ef = [oracle.rel_err(gf[q], fs[2, q]) for q in range(8)]
    ew = [oracle.rel_err(gw[q], ws[2, q]) for q in range(8)]
    ul = [float(np.nanmax(oracle.ulps(gf[q], fs[2, q]))) for q in range(8)]
    say(f"  f rel err  : " + " ".join("%.2e" % e for e in ef))
    say(f"  w rel err  : " + " ".join("%.2e" % e for e in ew))
    say(f"  f max ulps : " + " ".join("%.0f" % u for u in ul))
    return ef, ew, ul


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_large_domain_sampled(mhd, prec):
    ef, ew, _ = _sampled_full_step(mhd, "large1024x512x512", prec)
    if prec == "f64":
        assert max(ef) <= TOL_F64 and max(ew) <= TOL_F64
    else:
        amp = inputs.WORKLOADS["large1024x512x512"]["amp"]
        for q in range(8):
            assert ef[q] <= (TOL_F32C_1 if amp[q] > 0 else TOL_F32C_1_FROM_ZERO), q


@pytest.mark.parametrize("prec", ["f64", "f32c"])
def test_paper_benchmark_state_sampled(mhd, prec):
    ef, ew, _ = _sampled_full_step(mhd, "w0_512", prec)
    if prec == "f64":
        assert max(ef) <= TOL_F64 and max(ew) <= TOL_F64
    else:
        assert max(ef) <= TOL_F32C_W0


def _run_512(mhd, f0, prec, nsteps, dt):
    import torch
    S = mhd.Solver(512, 512, 512, prec)
    bufs = [S.upload(f0), S.empty()]
    w = S.empty()
    comp = S.zeros() if prec == "f32c" else None
    cur = S.step(bufs, 0, w, comp, dt, nsteps)
    torch.cuda.synchronize()
    out = S.interior_view(bufs[cur])
    del bufs[1 - cur], w, comp
    return S, out


@pytest.mark.parametrize("nsteps", [1, 100])
def test_f32_storage_against_gpu_f64_512(mhd, nsteps):
    """Per-field error of FP32C (and of the plain-FP32 ablation) against
    the FP64 path at 512^3, every interior cell."""
    wl = inputs.WORKLOADS["prec512"]
    f0 = inputs.workload_state("prec512").astype(np.float32).astype(np.float64)
    S64, ref = _run_512(mhd, f0, "f64", nsteps, wl["dt"])
    refs = [ref[q].cpu().numpy() for q in range(8)]
    S64.close()
    del ref
    out = {}
    for prec in ("f32c", "f32"):
        S, got = _run_512(mhd, f0, prec, nsteps, wl["dt"])
        out[prec] = [oracle.rel_err(got[q].cpu().double().numpy(), refs[q]) for q in range(8)]
        say(f"512^3 {prec} vs GPU f64, {nsteps} step(s): " +
            " ".join("%.2e" % e for e in out[prec]))
        S.close()
        del got
    if nsteps == 1:
        assert max(out["f32c"]) <= TOL_F32C_512_1
    else:
        assert max(out["f32c"]) <= TOL_F32C_512_100
        assert max(out["f32"]) <= TOL_F32_512_100
        # over 100 steps the compensated path is the more accurate one on
        # every field
        assert all(c < p for c, p in zip(out["f32c"], out["f32"]))

"""The C-ABI library loads on the CPU and exports every declared symbol;
argument validation and the no-device path return the documented codes.
No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2103_01597_amd import mhd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"^\s*(?:void|int|int64_t|const char)\s*\*?\s*(mhd\w*)\s*\(",
                                 text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(mhd.LIB_PATH):
        pytest.fail("libmhd.so is not built (run __graft_entry__.build())")
    return mhd.lib()


def test_every_declared_symbol_is_exported(L):
    from paper_2103_01597_amd import nn
    declared = _declared("mhd.h") + _declared("mhdnn.h")
    assert set(_declared("mhd.h")) == set(mhd.EXPORTS)
    assert set(_declared("mhdnn.h")) == set(nn.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", mhd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (\w+)$", out, re.M))
    for name in declared:
        assert name in exported, name
        assert getattr(L, name) is not None


def test_strerror_and_defaults(L):
    assert L.mhd_strerror(0) == b"ok"
    assert L.mhd_strerror(1) == b"invalid argument"
    assert L.mhd_strerror(2) == b"no usable HIP device"
    assert L.mhd_strerror(99) == b"unknown status"
    cfg = mhd.Config()
    L.mhd_config_default(ctypes.byref(cfg), 32, 16, 8, mhd.F32C)
    assert (cfg.nx, cfg.ny, cfg.nz, cfg.precision) == (32, 16, 8, 1)
    assert cfg.gamma == 5.0 / 3.0 and cfg.nu == 5e-3 and cfg.eta == 5e-3 and cfg.K == 5e-3
    assert cfg.cs0 == 1.0 and cfg.cp == 1.0 and cfg.mu0 == 1.0 and cfg.zeta == 0.0
    assert cfg.heat == 0.0 and cfg.cool == 0.0
    assert cfg.kernel == 3 and cfg.order == 6  # MHD_KERNEL_AUTO, sixth order
    assert abs(cfg.lx - 6.283185307179586) < 1e-15 and list(cfg.bext) == [0.0, 0.0, 0.0]
    L.mhd_config_default(ctypes.byref(cfg), 8, 8, 8, mhd.F64)
    assert cfg.kernel == 3 and cfg.order == 6


def test_segment_count_of_null_context(L):
    L.mhd_halo_segment_elems.restype = ctypes.c_int64
    L.mhd_halo_segment_elems.argtypes = [ctypes.c_void_p]
    assert L.mhd_halo_segment_elems(None) == -1


def _init(L, **kw):
    cfg = mhd.Config()
    L.mhd_config_default(ctypes.byref(cfg), 8, 8, 8, 0)
    for k, v in kw.items():
        setattr(cfg, k, v)
    ctx = ctypes.c_void_p(12345)
    lay = mhd.Layout()
    rc = L.mhd_init(ctypes.byref(cfg), ctypes.byref(ctx), ctypes.byref(lay))
    return rc, ctx


@pytest.mark.parametrize("bad", [dict(nx=0), dict(ny=-3), dict(precision=3), dict(precision=-1),
                                 dict(gamma=1.0), dict(cp=0.0), dict(mu0=0.0),
                                 dict(lx=float("nan")), dict(lz=-1.0), dict(nu=float("inf")),
                                 dict(nx=3000, ny=3000, nz=3000), dict(kernel=4),
                                 dict(kernel=-1), dict(order=5), dict(order=0), dict(order=10),
                                 dict(heat=float("inf")), dict(cool=float("nan")),
                                 # 1023^3 FP32 cells fit a 4 GiB field, 1025^3 do not
                                 dict(nx=1017, ny=1017, nz=1017, precision=2, order=8)])
def test_init_rejects_invalid_config(L, bad):
    rc, ctx = _init(L, **bad)
    assert rc == 1
    assert ctx.value is None  # *out is NULL on failure


def test_null_arguments(L):
    vp = ctypes.c_void_p
    assert L.mhd_init(None, ctypes.byref(vp()), ctypes.byref(mhd.Layout())) == 1
    assert L.mhd_halo_periodic(None, vp(1), None) == 1
    assert L.mhd_rk3_substep(None, 0, vp(1), vp(2), vp(3), None, 1e-3, None) == 1
    cur = ctypes.c_int32(0)
    arr = (vp * 2)(1, 2)
    assert L.mhd_step(None, arr, ctypes.byref(cur), vp(3), None, 1e-3, 1, None) == 1
    out = ctypes.c_double()
    assert L.mhd_reduce(None, vp(1), 0, 0, ctypes.byref(out), None) == 1
    box = mhd.Box(0, 1, 0, 1, 0, 1)
    assert L.mhd_rk3_substep_box(None, 0, ctypes.byref(box), vp(1), vp(2), vp(3), None, 1e-3,
                                 None) == 1
    assert L.mhd_halo_pack(None, vp(1), vp(2), None) == 1
    assert L.mhd_halo_unpack(None, vp(1), vp(2), None) == 1
    assert L.mhd_halo_exchange_self(None, vp(1), vp(2), vp(3), None) == 1
    assert L.mhd_step_segmented(None, arr, ctypes.byref(cur), vp(3), None, 1e-3, 1, vp(4), vp(5),
                                None, None) == 1
    L.mhd_finalize(None)


def test_bandwidth_probe_validation(L):
    """Invalid probe arguments are rejected before anything is launched."""
    vp = ctypes.c_void_p
    assert L.mhd_bandwidth_probe(4, vp(16), vp(32), vp(48), 1 << 20, None) == 1
    assert L.mhd_bandwidth_probe(-1, vp(16), vp(32), vp(48), 1 << 20, None) == 1
    assert L.mhd_bandwidth_probe(0, None, None, vp(48), 1 << 20, None) == 1
    assert L.mhd_bandwidth_probe(0, vp(16), None, None, 1 << 20, None) == 1
    assert L.mhd_bandwidth_probe(0, vp(16), None, vp(48), 1000, None) == 1  # not 16-byte units
    assert L.mhd_bandwidth_probe(1, vp(16), None, vp(48), 0, None) == 1
    assert L.mhd_bandwidth_probe(2, vp(16), None, vp(48), 1 << 20, None) == 1  # triad needs b
    assert L.mhd_bandwidth_probe(3, vp(16), vp(48), vp(48), 1 << 20, None) == 1  # b aliases c
    assert L.mhd_bandwidth_probe(0, vp(48), None, vp(48), 1 << 20, None) == 1  # a aliases c


@pytest.mark.parametrize("ok", [dict(), dict(order=2), dict(order=8, kernel=1),
                                dict(order=8, kernel=0), dict(order=4, kernel=2),
                                dict(order=2, kernel=2), dict(order=8, kernel=2, precision=1),
                                dict(order=8, kernel=2, precision=0),
                                dict(nx=1017, ny=1017, nz=1017, precision=2, order=6)])
def test_no_device_path(L, ok):
    """A valid configuration gets past validation to the device query:
    without a GPU init reports MHD_ERR_DEVICE, with one it succeeds."""
    rc, ctx = _init(L, **ok)
    if rc == 0:
        assert ctx.value is not None
        L.mhd_finalize(ctx)
        return
    assert rc == 2
    assert ctx.value is None

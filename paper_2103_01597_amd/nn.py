"""Python binding of the closure ABI (include/mhdnn.h): argument marshalling.

Every computation runs in libmhd.so's HIP kernels; torch tensors provide the
device memory (BF16 activations are torch.bfloat16 tensors, whose storage is
the raw 16-bit pattern the kernels read and write).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import mhd as _mhd

EXPORTS = ("mhdnn_box_filter4", "mhdnn_pack", "mhdnn_conv3d_fwd", "mhdnn_conv3d_dgrad",
           "mhdnn_wgrad_workspace_floats", "mhdnn_conv3d_wgrad", "mhdnn_prepare_weights",
           "mhdnn_mse", "mhdnn_pair", "mhdnn_field_stats_workspace_doubles",
           "mhdnn_field_stats", "mhdnn_adam", "mhdnn_apply", "mhdnn_conv3d_wgrad_noalloc")
_INT64_RESULT = ("mhdnn_wgrad_workspace_floats", "mhdnn_field_stats_workspace_doubles")
LAYERS = ((8, 32, True), (32, 32, True), (32, 8, False))  # (cin, cout, gelu)

_bound = False


def lib():
    global _bound
    L = _mhd.lib()
    if _bound:
        return L
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    fp = ctypes.POINTER(ctypes.c_float)
    L.mhdnn_box_filter4.argtypes = [vp, vp, vp, vp]
    L.mhdnn_pack.argtypes = [vp, vp, i64, i64, i64, i64, i64, i32, i32, fp, fp, vp, vp]
    L.mhdnn_conv3d_fwd.argtypes = [vp, vp, vp, i32, i32, i32, i32, i32, vp, vp, vp, vp]
    L.mhdnn_conv3d_dgrad.argtypes = [vp, vp, vp, i32, i32, i32, i32, vp, vp]
    L.mhdnn_wgrad_workspace_floats.argtypes = [i32, i32]
    L.mhdnn_wgrad_workspace_floats.restype = i64
    L.mhdnn_conv3d_wgrad.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp, vp]
    L.mhdnn_conv3d_wgrad_noalloc.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp]
    L.mhdnn_prepare_weights.argtypes = [vp, i32, i32, vp, vp, vp]
    L.mhdnn_mse.argtypes = [vp, vp, fp, i32, i32, vp, vp, vp]
    L.mhdnn_pair.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.mhdnn_field_stats_workspace_doubles.argtypes = []
    L.mhdnn_field_stats_workspace_doubles.restype = i64
    L.mhdnn_field_stats.argtypes = [vp, i64, i64, vp, vp, vp]
    L.mhdnn_adam.argtypes = [vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
    L.mhdnn_apply.argtypes = [vp, vp, vp, vp, fp, vp, vp]
    for fn in EXPORTS:
        if fn not in _INT64_RESULT:
            getattr(L, fn).restype = ctypes.c_int
    _bound = True
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _st(stream=None):
    return _mhd._stream(stream)


def _chk(fn, rc):
    if rc != 0:
        raise _mhd.MhdError(fn, rc)


def _f8(vals):
    return (ctypes.c_float * 8)(*[float(v) for v in vals])


def box_filter4(solver, fine, coarse, stream=None):
    _chk("mhdnn_box_filter4", lib().mhdnn_box_filter4(solver._ctx, _p(fine), _p(coarse), _st(stream)))


def pack(src, n, batch, mean, inv_std, out, *, sub=None, batch_stride=None, field_stride=None,
         origin=0, row=None, plane=None, stream=None):
    n3 = n ** 3
    _chk("mhdnn_pack", lib().mhdnn_pack(
        _p(src), _p(sub), 8 * n3 if batch_stride is None else batch_stride,
        n3 if field_stride is None else field_stride, origin, n if row is None else row,
        n * n if plane is None else plane, n, batch, _f8(mean), _f8(inv_std), _p(out), _st(stream)))


def pack_solver(solver, fields, mean, inv_std, out, sub=None, stream=None):
    L = solver.layout
    nx, ny, nz = solver.n
    assert nx == ny == nz
    pack(fields, nx, 1, mean, inv_std, out, sub=sub, batch_stride=0, field_stride=L.field_stride,
         origin=L.interior_offset, row=L.mx, plane=L.mx * L.my, stream=stream)


def conv3d_fwd(x, w_pad, bias, n, batch, cin, cout, mode, z=None, a=None, y=None, stream=None):
    _chk("mhdnn_conv3d_fwd", lib().mhdnn_conv3d_fwd(_p(x), _p(w_pad), _p(bias), n, batch, cin, cout,
                                                    mode, _p(z), _p(a), _p(y), _st(stream)))


def conv3d_dgrad(dz, wt_pad, zprev, n, batch, cin_dz, cprev, dprev, stream=None):
    _chk("mhdnn_conv3d_dgrad", lib().mhdnn_conv3d_dgrad(_p(dz), _p(wt_pad), _p(zprev), n, batch,
                                                        cin_dz, cprev, _p(dprev), _st(stream)))


def wgrad_workspace_floats(n, batch):
    return int(lib().mhdnn_wgrad_workspace_floats(n, batch))


def conv3d_wgrad(x, dz, n, batch, cin, cout, workspace, dw, db, stream=None):
    _chk("mhdnn_conv3d_wgrad", lib().mhdnn_conv3d_wgrad(_p(x), _p(dz), n, batch, cin, cout,
                                                        _p(workspace), _p(dw), _p(db), _st(stream)))


def prepare_weights(w, cin, cout, w_pad, wt_pad=None, stream=None):
    _chk("mhdnn_prepare_weights", lib().mhdnn_prepare_weights(_p(w), cin, cout, _p(w_pad),
                                                              _p(wt_pad), _st(stream)))


def mse(y, target, tscale, n, batch, dy, partials, stream=None):
    """target: field-major [batch][8][n^3] FP32, scaled per field by tscale."""
    _chk("mhdnn_mse", lib().mhdnn_mse(_p(y), _p(target), _f8(tscale), n, batch, _p(dy),
                                      _p(partials), _st(stream)))


def pair(coarse_solver, stepped, c_now, c_next, x_out, d_out, stream=None):
    _chk("mhdnn_pair", lib().mhdnn_pair(coarse_solver._ctx, _p(stepped), _p(c_now), _p(c_next),
                                        _p(x_out), _p(d_out), _st(stream)))


def field_stats(x, npairs, n3, stream=None):
    """Per-field (mean, std) of samples [npairs][8][n3] as host float64 arrays."""
    import torch
    ws = torch.empty(int(lib().mhdnn_field_stats_workspace_doubles()), dtype=torch.float64,
                     device=x.device)
    out = torch.empty(16, dtype=torch.float64, device=x.device)
    _chk("mhdnn_field_stats", lib().mhdnn_field_stats(_p(x), npairs, n3, _p(ws), _p(out),
                                                      _st(stream)))
    host = out.cpu().numpy()
    return host[:8].copy(), host[8:].copy()


def adam(p, g, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    _chk("mhdnn_adam", lib().mhdnn_adam(_p(p), _p(g), _p(m), _p(v), p.numel(), lr, b1, b2, eps, t,
                                        _st(stream)))


def apply(solver, fields, comp, y, scale, guard=None, stream=None):
    """guard: optional int32 device tensor of 2 elements (see mhdnn.h)."""
    _chk("mhdnn_apply", lib().mhdnn_apply(solver._ctx, _p(fields), _p(comp), _p(y), _f8(scale),
                                          _p(guard), _st(stream)))


class Closure:
    """The 8->32->32->8 periodic conv net with FP32 master weights, BF16
    kernel weights and Adam state, all on the GPU."""

    def __init__(self, seed=0, device="cuda"):
        import torch
        rng = np.random.default_rng(seed)
        self.w, self.b, self.m, self.v = [], [], [], []
        self.w_pad, self.wt_pad = [], []
        for cin, cout, _ in LAYERS:
            std = math.sqrt(2.0 / (27 * cin))
            w = torch.from_numpy(rng.standard_normal((cout, 27, cin)) * std).float().to(device)
            self.w.append(w)
            self.b.append(torch.zeros(cout, device=device))
            self.w_pad.append(torch.empty(32 * 27 * cin, dtype=torch.bfloat16, device=device))
            self.wt_pad.append(torch.empty(32 * 27 * cout, dtype=torch.bfloat16, device=device))
        self.params = [t for pair in zip(self.w, self.b) for t in pair]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.t = 0
        self.refresh()

    def refresh(self):
        for (cin, cout, _), w, wp, wt in zip(LAYERS, self.w, self.w_pad, self.wt_pad):
            prepare_weights(w, cin, cout, wp, wt)

    def forward(self, x, n, batch):
        """x: BF16 [batch*n^3*8]; returns FP32 y [batch*n^3*8] and the cache."""
        import torch
        dev = x.device
        cells = batch * n ** 3
        cache = [x]
        h = x
        for i, (cin, cout, act) in enumerate(LAYERS):
            if act:
                z = torch.empty(cells * cout, dtype=torch.bfloat16, device=dev)
                a = torch.empty_like(z)
                conv3d_fwd(h, self.w_pad[i], self.b[i], n, batch, cin, cout, 0, z=z, a=a)
                cache += [z, a]
                h = a
            else:
                y = torch.empty(cells * cout, dtype=torch.float32, device=dev)
                conv3d_fwd(h, self.w_pad[i], self.b[i], n, batch, cin, cout, 1, y=y)
        return y, cache

    def backward(self, cache, dy, n, batch, workspace=None):
        """dy: BF16 gradient of the output; returns [dW1, db1, dW2, db2, dW3, db3]."""
        import torch
        dev = dy.device
        cells = batch * n ** 3
        x, z1, a1, z2, a2 = cache
        if workspace is None:
            workspace = torch.empty(wgrad_workspace_floats(n, batch), device=dev)
        grads = [None] * 6
        ins = [x, a1, a2]
        zs = [None, z1, z2]
        g = dy
        for i in reversed(range(3)):
            cin, cout, _ = LAYERS[i]
            dw = torch.empty(cout * 27 * cin, device=dev)
            db = torch.empty(cout, device=dev)
            conv3d_wgrad(ins[i], g, n, batch, cin, cout, workspace, dw, db)
            grads[2 * i], grads[2 * i + 1] = dw.view(cout, 27, cin), db
            if i > 0:
                d = torch.empty(cells * cin, dtype=torch.bfloat16, device=dev)
                conv3d_dgrad(g, self.wt_pad[i], zs[i], n, batch, cout, cin, d)
                g = d
        return grads

    def step(self, grads, lr):
        self.t += 1
        for p, g, m, v in zip(self.params, grads, self.m, self.v):
            adam(p, g.contiguous(), m, v, lr, self.t)
        self.refresh()

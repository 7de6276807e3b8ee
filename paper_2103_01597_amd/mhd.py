"""Python binding of libmhd.so (include/mhd.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels.  PyTorch serves
as the device allocator and supplies the stream (the current torch stream
unless one is passed).  If the library is not built, :func:`lib` raises --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhd.so")

F64, F32C, F32 = 0, 1, 2
PRECISIONS = {"f64": F64, "f32c": F32C, "f32": F32}
KERNELS = {"tiled": 0, "direct": 1, "split": 2, "auto": 3}
RED_OPS = {"sum": 0, "sumsq": 1, "maxabs": 2, "min": 3, "max": 4, "sumexp": 5, "nonfinite": 6}
FIELD_NAMES = ("lnrho", "ux", "uy", "uz", "ss", "ax", "ay", "az")
STATUS = {0: "MHD_OK", 1: "MHD_ERR_INVALID", 2: "MHD_ERR_NO_DEVICE", 3: "MHD_ERR_DEVICE",
          4: "MHD_ERR_NOMEM"}

# every symbol declared in include/mhd.h
EXPORTS = ("mhd_config_default", "mhd_init", "mhd_finalize", "mhd_strerror",
           "mhd_halo_periodic", "mhd_rk3_substep", "mhd_step", "mhd_halo_segment_elems",
           "mhd_halo_pack", "mhd_halo_unpack", "mhd_halo_exchange_self", "mhd_rk3_substep_box",
           "mhd_step_segmented", "mhd_reduce", "mhd_bandwidth_probe")
BW_KINDS = {"copy": 0, "copy_nt": 1, "triad": 2, "triad_nt": 3}


class Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("order", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("cs0", ctypes.c_double), ("gamma", ctypes.c_double), ("cp", ctypes.c_double),
                ("lnrho0", ctypes.c_double), ("mu0", ctypes.c_double), ("nu", ctypes.c_double),
                ("zeta", ctypes.c_double), ("eta", ctypes.c_double), ("K", ctypes.c_double),
                ("bext", ctypes.c_double * 3), ("heat", ctypes.c_double),
                ("cool", ctypes.c_double)]


class Layout(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("mx", "my", "mz", "field_stride", "elem_size", "interior_offset", "total_elems",
                 "halo", "kernel")]


class Box(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("x0", "x1", "y0", "y1", "z0", "z1")]


class MhdError(RuntimeError):
    def __init__(self, fn, rc):
        super().__init__(f"{fn} failed: {STATUS.get(rc, rc)}")
        self.rc = rc


_lib = None


def lib():
    """Load libmhd.so (built by ``__graft_entry__.build()``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.mhd_config_default.argtypes = [ctypes.POINTER(Config), i32, i32, i32, i32]
    L.mhd_config_default.restype = None
    L.mhd_init.argtypes = [ctypes.POINTER(Config), ctypes.POINTER(vp), ctypes.POINTER(Layout)]
    L.mhd_finalize.argtypes = [vp]
    L.mhd_finalize.restype = None
    L.mhd_strerror.argtypes = [ctypes.c_int]
    L.mhd_strerror.restype = ctypes.c_char_p
    L.mhd_halo_periodic.argtypes = [vp, vp, vp]
    L.mhd_rk3_substep.argtypes = [vp, i32, vp, vp, vp, vp, dbl, vp]
    L.mhd_step.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i32), vp, vp, dbl, i32, vp]
    L.mhd_reduce.argtypes = [vp, vp, i32, i32, ctypes.POINTER(dbl), vp]
    L.mhd_halo_segment_elems.argtypes = [vp]
    L.mhd_halo_segment_elems.restype = ctypes.c_int64
    L.mhd_halo_pack.argtypes = [vp, vp, vp, vp]
    L.mhd_halo_unpack.argtypes = [vp, vp, vp, vp]
    L.mhd_halo_exchange_self.argtypes = [vp, vp, vp, vp, vp]
    L.mhd_rk3_substep_box.argtypes = [vp, i32, ctypes.POINTER(Box), vp, vp, vp, vp, dbl, vp]
    L.mhd_step_segmented.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(i32), vp, vp, dbl,
                                     i32, vp, vp, vp, vp]
    L.mhd_bandwidth_probe.argtypes = [i32, vp, vp, vp, ctypes.c_int64, vp]
    for fn in ("mhd_init", "mhd_halo_periodic", "mhd_rk3_substep", "mhd_step", "mhd_reduce",
               "mhd_halo_pack", "mhd_halo_unpack", "mhd_halo_exchange_self",
               "mhd_rk3_substep_box", "mhd_step_segmented", "mhd_bandwidth_probe"):
        getattr(L, fn).restype = ctypes.c_int
    _lib = L
    return L


def _check(fn, rc):
    if rc != 0:
        raise MhdError(fn, rc)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One context of the library on the current HIP device.

    Buffers are flat torch tensors of ``layout.total_elems`` elements; use
    :meth:`grid_view` / :meth:`interior_view` for (8, mz, my, mx) views.
    """

    def __init__(self, nx, ny, nz, precision="f64", kernel=None, order=6, **phys):
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        cfg = Config()
        lib().mhd_config_default(ctypes.byref(cfg), nx, ny, nz, self.precision)
        cfg.order = int(order)
        if kernel is not None:  # None: the library picks (MHD_KERNEL_AUTO)
            cfg.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
        for k, v in phys.items():
            if k == "bext":
                cfg.bext = (ctypes.c_double * 3)(*[float(b) for b in v])
            elif k == "lengths":
                cfg.lx, cfg.ly, cfg.lz = (float(x) for x in v)
            else:
                setattr(cfg, k, float(v))
        self.cfg = cfg
        self.layout = Layout()
        self._ctx = ctypes.c_void_p()
        _check("mhd_init", lib().mhd_init(ctypes.byref(cfg), ctypes.byref(self._ctx),
                                          ctypes.byref(self.layout)))
        self.n = (nx, ny, nz)
        self.order = int(order)
        self.r = int(self.layout.halo)
        self.kernel = {v: k for k, v in KERNELS.items()}[int(self.layout.kernel)]

    def close(self):
        self._segbufs = None
        if self._ctx:
            lib().mhd_finalize(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- buffers
    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.layout.elem_size == 8 else torch.float32

    def empty(self):
        import torch
        return torch.empty(self.layout.total_elems, dtype=self.torch_dtype, device="cuda")

    def zeros(self):
        import torch
        return torch.zeros(self.layout.total_elems, dtype=self.torch_dtype, device="cuda")

    def grid_view(self, buf):
        L = self.layout
        return buf.as_strided((8, L.mz, L.my, L.mx), (L.field_stride, L.my * L.mx, L.mx, 1))

    def interior_view(self, buf):
        nx, ny, nz = self.n
        r = self.r
        return self.grid_view(buf)[:, r:r + nz, r:r + ny, r:r + nx]

    def upload(self, fields: np.ndarray, buf=None, fill_halo=True):
        """Copy an (8, nz, ny, nx) host array into the interior of a buffer
        (converted to the storage type) and fill its periodic halo."""
        import torch
        buf = self.empty() if buf is None else buf
        host = torch.from_numpy(np.ascontiguousarray(fields)).to(self.torch_dtype)
        self.interior_view(buf).copy_(host)
        if fill_halo:
            self.halo_periodic(buf)
        return buf

    def upload_fields(self, fields, buf=None, fill_halo=True):
        """Like ``upload`` from an iterable of (q, (nz, ny, nx) host array),
        one field at a time (e.g. ``inputs.fourier_mode_fields``)."""
        import torch
        buf = self.empty() if buf is None else buf
        view = self.interior_view(buf)
        for q, f in fields:
            view[q].copy_(torch.from_numpy(np.ascontiguousarray(f)).cuda().to(self.torch_dtype))
        if fill_halo:
            self.halo_periodic(buf)
        return buf

    def download(self, buf) -> np.ndarray:
        """Interior of a buffer as an (8, nz, ny, nx) float64 host array."""
        return self.interior_view(buf).cpu().double().numpy()

    # -------------------------------------------------------------- ABI
    def halo_periodic(self, buf, stream=None):
        _check("mhd_halo_periodic", lib().mhd_halo_periodic(self._ctx, _ptr(buf), _stream(stream)))

    def rk3_substep(self, s, f_in, f_out, w, comp=None, dt=1e-3, stream=None):
        _check("mhd_rk3_substep", lib().mhd_rk3_substep(self._ctx, s, _ptr(f_in), _ptr(f_out),
                                                        _ptr(w), _ptr(comp), dt, _stream(stream)))

    def step(self, f, cur, w, comp=None, dt=1e-3, nsteps=1, stream=None) -> int:
        """nsteps RK3 steps starting from f[cur]; returns the result's index."""
        arr = (ctypes.c_void_p * 2)(f[0].data_ptr(), f[1].data_ptr())
        c = ctypes.c_int32(cur)
        _check("mhd_step", lib().mhd_step(self._ctx, arr, ctypes.byref(c), _ptr(w), _ptr(comp),
                                          dt, nsteps, _stream(stream)))
        return c.value

    # ---------------------------------------------- segmented iteration
    def halo_segment_elems(self) -> int:
        return int(lib().mhd_halo_segment_elems(self._ctx))

    def segment_buffer(self):
        import torch
        return torch.empty(self.halo_segment_elems(), dtype=self.torch_dtype, device="cuda")

    def halo_pack(self, fields, sendbuf, stream=None):
        _check("mhd_halo_pack", lib().mhd_halo_pack(self._ctx, _ptr(fields), _ptr(sendbuf),
                                                    _stream(stream)))

    def halo_unpack(self, recvbuf, fields, stream=None):
        _check("mhd_halo_unpack", lib().mhd_halo_unpack(self._ctx, _ptr(recvbuf), _ptr(fields),
                                                        _stream(stream)))

    def halo_exchange_self(self, fields, sendbuf, recvbuf, stream=None):
        _check("mhd_halo_exchange_self",
               lib().mhd_halo_exchange_self(self._ctx, _ptr(fields), _ptr(sendbuf), _ptr(recvbuf),
                                            _stream(stream)))

    def rk3_substep_box(self, s, box, f_in, f_out, w, comp=None, dt=1e-3, stream=None):
        """box: (x0, x1, y0, y1, z0, z1) in interior cell indices, half-open."""
        b = Box(*[int(v) for v in box])
        _check("mhd_rk3_substep_box",
               lib().mhd_rk3_substep_box(self._ctx, s, ctypes.byref(b), _ptr(f_in), _ptr(f_out),
                                         _ptr(w), _ptr(comp), dt, _stream(stream)))

    def step_segmented(self, f, cur, w, comp=None, dt=1e-3, nsteps=1, sendbuf=None,
                       recvbuf=None, stream=None, comm_stream=None) -> int:
        """mhd_step with the inner/outer split and the packed halo exchange on
        comm_stream; returns the result's index.  Without explicit buffers the
        solver's own pair is used (allocated once and kept, so that no buffer
        is freed while queued work may still use it)."""
        arr = (ctypes.c_void_p * 2)(f[0].data_ptr(), f[1].data_ptr())
        c = ctypes.c_int32(cur)
        if sendbuf is None or recvbuf is None:
            if getattr(self, "_segbufs", None) is None:
                self._segbufs = (self.segment_buffer(), self.segment_buffer())
            sendbuf = self._segbufs[0] if sendbuf is None else sendbuf
            recvbuf = self._segbufs[1] if recvbuf is None else recvbuf
        _check("mhd_step_segmented",
               lib().mhd_step_segmented(self._ctx, arr, ctypes.byref(c), _ptr(w), _ptr(comp), dt,
                                        nsteps, _ptr(sendbuf), _ptr(recvbuf), _stream(stream),
                                        _stream(comm_stream)))
        return c.value

    def reduce(self, buf, field, op, stream=None) -> float:
        q = FIELD_NAMES.index(field) if isinstance(field, str) else int(field)
        out = ctypes.c_double()
        _check("mhd_reduce", lib().mhd_reduce(self._ctx, _ptr(buf), q, RED_OPS[op],
                                              ctypes.byref(out), _stream(stream)))
        return out.value


def bandwidth_probe(kind, a, b, c, stream=None):
    """One launch of a streaming kernel (``BW_KINDS``) over the byte size
    of ``c`` (flat device tensors; ``b`` is unused by the copies)."""
    nbytes = c.numel() * c.element_size()
    _check("mhd_bandwidth_probe", lib().mhd_bandwidth_probe(BW_KINDS[kind], _ptr(a), _ptr(b),
                                                            _ptr(c), nbytes, _stream(stream)))

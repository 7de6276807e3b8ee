"""mhdnn_conv3d_wgrad_noalloc (the weight gradient for callers that cannot
allocate) against mhdnn_conv3d_wgrad with a caller workspace: the same
kernels in the same order, so the results must agree bit for bit.  Two
calls in a row share the library's device array, the second with a smaller
input; a size beyond the array is rejected and leaves the next call intact.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SHAPES = [(8, 32), (32, 32), (32, 8), (8, 8)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def nn():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2103_01597_amd import nn as m
    m.lib()
    return m


def _inputs(rng, n, batch, cin, cout):
    import torch
    cells = batch * n ** 3
    x = torch.from_numpy(rng.standard_normal(cells * cin)).float().cuda().to(torch.bfloat16)
    dz = torch.from_numpy(rng.standard_normal(cells * cout)).float().cuda().to(torch.bfloat16)
    return x, dz


def _noalloc(nn, x, dz, n, batch, cin, cout, dw, db):
    import torch
    L = nn.lib()
    return L.mhdnn_conv3d_wgrad_noalloc(ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(dz.data_ptr()), n, batch, cin, cout,
                                        ctypes.c_void_p(dw.data_ptr()),
                                        ctypes.c_void_p(db.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("cin,cout", SHAPES)
def test_noalloc_equals_workspace_entry(nn, cin, cout):
    import torch
    rng = np.random.default_rng(70 + cin + cout)
    for n, batch in ((64, 4), (32, 2)):  # the second call is smaller
        say(f"wgrad noalloc cin={cin} cout={cout} n={n} batch={batch}")
        x, dz = _inputs(rng, n, batch, cin, cout)
        ws = torch.empty(nn.wgrad_workspace_floats(n, batch), device="cuda")
        dw_ref = torch.empty(cout * 27 * cin, device="cuda")
        db_ref = torch.empty(cout, device="cuda")
        nn.conv3d_wgrad(x, dz, n, batch, cin, cout, ws, dw_ref, db_ref)
        dw = torch.full_like(dw_ref, float("nan"))
        db = torch.full_like(db_ref, float("nan"))
        assert _noalloc(nn, x, dz, n, batch, cin, cout, dw, db) == 0
        torch.cuda.synchronize()
        assert torch.equal(dw, dw_ref) and torch.equal(db, db_ref)


def test_noalloc_size_limit(nn):
    """Beyond the library's array (64^3 at batch 33) the call is refused with
    MHD_ERR_INVALID; the largest fitting batch and a later call still work."""
    import torch
    rng = np.random.default_rng(90)
    cin, cout = 8, 8
    limit = 512 * (27 * 32 * 32 + 32)  # MHDNN_WGRAD_SCRATCH_FLOATS of include/mhdnn.h
    assert nn.wgrad_workspace_floats(64, 32) <= limit < nn.wgrad_workspace_floats(64, 33)
    x, dz = _inputs(rng, 16, 1, cin, cout)  # the pointers are never read on refusal
    dw = torch.zeros(cout * 27 * cin, device="cuda")
    db = torch.zeros(cout, device="cuda")
    assert _noalloc(nn, x, dz, 64, 33, cin, cout, dw, db) == 1
    assert _noalloc(nn, x, dz, 16, 1, 8, 16, dw, db) == 1  # no such layer shape
    torch.cuda.synchronize()
    assert torch.count_nonzero(dw).item() == 0  # nothing was launched
    for n, batch in ((64, 32), (16, 1)):  # the largest fitting batch, then a small call
        xx, dd = _inputs(rng, n, batch, cin, cout)
        ws = torch.empty(nn.wgrad_workspace_floats(n, batch), device="cuda")
        dw_ref = torch.empty_like(dw)
        db_ref = torch.empty_like(db)
        nn.conv3d_wgrad(xx, dd, n, batch, cin, cout, ws, dw_ref, db_ref)
        assert _noalloc(nn, xx, dd, n, batch, cin, cout, dw, db) == 0
        torch.cuda.synchronize()
        assert torch.equal(dw, dw_ref) and torch.equal(db, db_ref)

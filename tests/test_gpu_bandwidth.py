"""GPU check of the streaming kernels behind the achievable-bandwidth figure
(mhd_bandwidth_probe): every element of the output is the copy or the FP64
triad c = a + 3 b of the inputs, for sizes that are not multiples of a
workgroup's 4096-byte share, and nothing past the given size is written."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mhd():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_2103_01597_amd import mhd as m
    m.lib()
    return m


@pytest.mark.parametrize("kind", ["copy", "copy_nt", "triad", "triad_nt"])
@pytest.mark.parametrize("n", [2, 4096, 4098, 1 << 20, (1 << 20) + 18])
def test_bandwidth_probe_results(mhd, kind, n):
    import torch
    rng = np.random.default_rng(n)
    # small dyadic values: 3 b and a + 3 b are exact in FP64, so the
    # expected triad needs no rounding model
    a_h = rng.integers(-1000, 1000, n).astype(np.float64) / 1024
    b_h = rng.integers(-1000, 1000, n).astype(np.float64) / 1024
    a = torch.from_numpy(a_h).cuda()
    b = torch.from_numpy(b_h).cuda()
    c_full = torch.full((n + 8,), 7.0, dtype=torch.float64, device="cuda")
    mhd.bandwidth_probe(kind, a, b, c_full[:n])
    torch.cuda.synchronize()
    got = c_full.cpu().numpy()
    want = a_h if kind.startswith("copy") else a_h + 3.0 * b_h
    assert np.array_equal(got[:n], want)
    assert np.all(got[n:] == 7.0)

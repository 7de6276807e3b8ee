"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, the CPU
oracle sweep and the source/flag hash that ties a traffic profile to the
kernel it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_oracle_sweep_structure():
    import bench
    from paper_2103_01597_amd import inputs
    res = bench.oracle_sweep(inputs, inputs.WORKLOADS["prec512"], sizes=(16,))
    threads = {r["threads"] for r in res["runs"]}
    assert 1 in threads and res["threads_available"] in threads
    for r in res["runs"]:
        assert r["n"] == 16 and r["seconds"] > 0.001
        # seconds are rounded to 1 ms and GCUPS to 1e-6
        expect = 3 * 16 ** 3 / r["seconds"] / 1e9
        assert abs(r["gcups"] - expect) <= expect * 0.0005 / (r["seconds"] - 0.0005) + 1e-6


def test_kernel_hash_covers_source_and_flags(monkeypatch):
    import bench
    from paper_2103_01597_amd import build as hip_build
    h_split, h_tiled = bench.kernel_source_hash("split"), bench.kernel_source_hash("tiled")
    assert h_split != h_tiled and len(h_split) == 64
    # the hash does not depend on where the repository lives
    flags = ["/elsewhere/include" if f.startswith("/") else f for f in hip_build.FLAGS]
    monkeypatch.setattr(hip_build, "FLAGS", flags)
    assert bench.kernel_source_hash("split") == h_split
    # but it does depend on the kernel's own compile flags
    monkeypatch.setitem(hip_build.PER_FILE, "rk3_split.hip", ["-O2"])
    assert bench.kernel_source_hash("split") != h_split

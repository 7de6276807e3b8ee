#!/usr/bin/env python3
"""Throughput of the fused sixth-order MHD RK3 path on one MI355X.

Metric: GCUPS per RK3 substep = 3 * (interior cells) * steps / time / 1e9,
for FP64 (the headline `value`) and for FP32 storage with the compensated
update (reported beside it), on the 512^3 precision-comparison workload:
8 fields initialised as 1e-2 * (sum of 4 seeded Fourier modes, |k| <= 8),
cs0 = 1, gamma = 5/3, nu = eta = chi = 5e-3, dt = 1e-3, periodic halo
filled before every substep.  Inputs are resident in HBM before timing.

One timed step = 3 x (halo fill + fused RHS/RK3 substep), exactly the
launch sequence of mhd_step.  HIP events on the launch stream bracket the
whole timed region and every fused-substep launch; the per-launch average
gives the roofline entry of the dominant kernel.

`--gpus N` with N > 1 exits: the path is one GPU's share of the domain and
has no multi-GPU mode.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# translation units each fused kernel is built from (the _dflt and _f64r3
# units include the kernel file and build some of its instantiations)
KERNEL_SOURCE = {"split": ("rk3_split.hip", "rk3_split_f64r3.hip", "rk3_split_dflt.hip"),
                 "tiled": ("rk3_tiled.hip", "rk3_tiled_dflt.hip"), "direct": ("rk3_direct.hip",)}
KERNEL_SYMBOL = {"split": "k_rk3_split", "tiled": "k_rk3_tiled", "direct": "k_rk3_direct"}

WORKLOAD_TEXT = {
    "prec512": "prec512: 512^3 periodic, 8 fields, 1e-2 x 4 Fourier modes |k|<=8 seed 3, "
               "dt 1e-3, halo fill every substep",
    "sub256": "sub256: 256^3 periodic, 8 fields, 1e-2 x 4 Fourier modes |k|<=8 seed 2, "
              "dt 1e-3, halo fill every substep",
    "w0_512": "w0: 512^3 periodic, 8 fields i.i.d. U[0,1) (the paper's benchmark state), "
              "dt 2^-23, halo fill every substep",
    "large1024x512x512": "large: 1024x512x512 periodic (4pi x 2pi x 2pi), u modes |k|<=16 "
                         "amp 0.1, A amp 1e-3, seed 4, dt 1e-3, halo fill every substep",
}

# Compulsory HBM bytes per interior cell of the fused substep (8 fields):
# read f_in, write w and f_out, plus read w for s > 0; F32C also reads and
# writes the compensation array.
BYTES_PER_CELL = {
    "f64": (3 * 8 * 8, 4 * 8 * 8, 4 * 8 * 8),   # 192, 256, 256
    "f32c": (5 * 8 * 4, 6 * 8 * 4, 6 * 8 * 4),  # 160, 192, 192
    "f32": (3 * 8 * 4, 4 * 8 * 4, 4 * 8 * 4),   # 96, 128, 128
}


def time_segmented(S, torch, bufs, cur, w, comp, dt, steps, cells):
    """The same steps through mhd_step_segmented (inner box on the launch
    stream, packed halo exchange on a second stream, outer shell after it)."""
    comm = torch.cuda.Stream()
    send, recv = S.segment_buffer(), S.segment_buffer()
    stream = torch.cuda.current_stream()
    cur = S.step_segmented(bufs, cur, w, comp, dt, 1, send, recv, comm_stream=comm)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    cur = S.step_segmented(bufs, cur, w, comp, dt, steps, send, recv, comm_stream=comm)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    return dict(ms_per_step=round(ms / steps, 4),
                gcups=round(3 * cells * steps / (ms * 1e-3) / 1e9, 4))


def achievable_bandwidth(mhd, torch, nbytes=2 << 30, launches=10):
    """Achievable HBM bandwidth: the library's plain copy and triad kernels
    (with and without non-temporal hints) over arrays of nbytes each, far
    larger than the last-level cache; GB/s = bytes read and written per
    launch / average launch time (HIP events on the launch stream)."""
    stream = torch.cuda.current_stream()
    a = torch.full((nbytes // 8,), 1.0, dtype=torch.float64, device="cuda")
    b = torch.full_like(a, 2.0)
    c = torch.empty_like(a)
    moved = {"copy": 2 * nbytes, "copy_nt": 2 * nbytes, "triad": 3 * nbytes, "triad_nt": 3 * nbytes}
    out = {}
    for kind in ("copy", "copy_nt", "triad", "triad_nt"):
        for _ in range(2):
            mhd.bandwidth_probe(kind, a, b, c)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(launches)]
        for e0, e1 in ev:
            e0.record(stream)
            mhd.bandwidth_probe(kind, a, b, c)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = sum(e0.elapsed_time(e1) for e0, e1 in ev) / launches
        out[kind] = round(moved[kind] / (ms * 1e-3) / 1e9, 1)
    ok = bool(torch.all(c == 7.0).item())  # the last launch was a triad: 1 + 3 * 2
    del a, b, c
    torch.cuda.empty_cache()
    best = max(out, key=out.get)
    return dict(gbs=out, best_kind=best, best_gbs=out[best], array_bytes=nbytes,
                launches=launches, result_ok=ok)


def order_study(mhd, inputs, torch, steps=5, warmup=1, name="sub256"):
    """Time per cell per RK3 step for the stencil orders 2, 4, 6 and 8 at
    256^3 (the single-GPU part of the paper's order study, Section 5), FP64
    and FP32C, each with the library's kernel for that order and precision
    (mhd_step, halo fill included)."""
    wl = inputs.WORKLOADS[name]
    n = wl["shape"]
    cells = math.prod(n)
    out = {"workload": WORKLOAD_TEXT[name], "steps": steps}
    for prec in ("f64", "f32c"):
        per = {}
        for order in (2, 4, 6, 8):
            S = mhd.Solver(*n, prec, order=order)
            bufs = [S.upload_fields(inputs.workload_fields(name)), S.empty()]
            w = S.zeros()
            comp = S.zeros() if prec == "f32c" else None
            cur = S.step(bufs, 0, w, comp, wl["dt"], warmup)
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            stream = torch.cuda.current_stream()
            t0.record(stream)
            cur = S.step(bufs, cur, w, comp, wl["dt"], steps)
            t1.record(stream)
            torch.cuda.synchronize()
            ms = t0.elapsed_time(t1) / steps
            nonfinite = S.reduce(bufs[cur], 0, "nonfinite")
            gbs = cells * sum(BYTES_PER_CELL[prec]) / (ms * 1e-3) / 1e9
            per[str(order)] = {"kernel": KERNEL_SYMBOL[S.kernel], "ms_per_step": round(ms, 4),
                               "ns_per_cell_step": round(ms * 1e6 / cells, 4),
                               "gcups": round(3 * cells / (ms * 1e-3) / 1e9, 3),
                               "roofline_frac": round(gbs / HBM_PEAK_GBS, 4),
                               "nonfinite": nonfinite}
            S.close()
            del bufs, w, comp
            torch.cuda.empty_cache()
            print(f"# order {order} {prec}: {json.dumps(per[str(order)])}", file=sys.stderr,
                  flush=True)
        out[prec] = per
    return out


def run_precision(mhd, inputs, torch, name, prec, steps, warmup, kernel, segmented=False,
                  repeats=5):
    wl = inputs.WORKLOADS[name]
    n = wl["shape"]
    cells = n[0] * n[1] * n[2]
    S = mhd.Solver(*n, prec, kernel, lengths=wl.get("lengths", (2 * math.pi,) * 3))
    kernel = S.kernel
    bufs = [S.upload_fields(inputs.workload_fields(name)), S.empty()]
    w = S.zeros()
    comp = S.zeros() if prec == "f32c" else None
    dt = wl["dt"]
    stream = torch.cuda.current_stream()
    cur = S.step(bufs, 0, w, comp, dt, warmup)
    torch.cuda.synchronize()

    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(3)] for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for k in range(steps):
        for s in range(3):
            S.halo_periodic(bufs[cur])
            ev[k][s][0].record(stream)
            S.rk3_substep(s, bufs[cur], bufs[1 - cur], w, comp, dt)
            ev[k][s][1].record(stream)
            cur ^= 1
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_time(t1)
    kern_ms = [[ev[k][s][0].elapsed_time(ev[k][s][1]) for s in range(3)] for k in range(steps)]
    sum_kern_ms = sum(sum(r) for r in kern_ms)
    alg_bytes = steps * cells * sum(BYTES_PER_CELL[prec])
    achieved = alg_bytes / (sum_kern_ms * 1e-3) / 1e9
    # repeats of the same K steps (mhd_step, the same launch sequence) for
    # the spread; the first region above is the reported one
    reps = [total_ms / steps]
    for _ in range(repeats - 1):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        cur = S.step(bufs, cur, w, comp, dt, steps)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1) / steps)
    nonfinite = S.reduce(bufs[cur], 0, "nonfinite")
    seg = time_segmented(S, torch, bufs, cur, w, comp, dt, steps, cells) if segmented else None
    res = dict(
        gcups=3 * cells * steps / (total_ms * 1e-3) / 1e9,
        ms_per_step=total_ms / steps,
        wall_s=wall,
        kernel_ms_avg=sum_kern_ms / (3 * steps),
        kernel_ms_by_substep=[sum(r[s] for r in kern_ms) / steps for s in range(3)],
        kernel_gbs=achieved,
        kernel_gcups=3 * cells * steps / (sum_kern_ms * 1e-3) / 1e9,
        nonfinite=nonfinite,
        kernel=kernel,
        segmented=seg,
        ms_per_step_repeats=[round(v, 4) for v in reps],
        median_gcups=3 * cells / (float(np.median(reps)) * 1e-3) / 1e9,
    )
    S.close()
    del bufs, w, comp
    torch.cuda.empty_cache()
    return res


def kernel_source_hash(kernel):
    """SHA-256 of the sources a fused kernel is built from (its own file and
    the headers it shares) and of its compile flags."""
    import hashlib
    from paper_2103_01597_amd import build as hip_build
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2103_01597_amd", "csrc")
    for name in (*KERNEL_SOURCE[kernel], "rk3_common.hpp", "mhd_internal.hpp"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    for unit in KERNEL_SOURCE[kernel]:
        flags = hip_build.FLAGS + hip_build.PER_FILE.get(unit, [])
        h.update(" ".join(f for f in flags if not f.startswith("/")).encode())
    return h.hexdigest()


def measured_traffic(kernel, prec, workload):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same counters on
    a copy kernel of known size), or None when there is none or the kernel's
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{KERNEL_SYMBOL[kernel]}_{prec}_{workload}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ": " in line:
                k, v = line[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash(kernel):
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(inputs, wl, n1=256):
    """The oracle as it stands, one RK3 step on an n1^3 grid of the same
    workload recipe (a bounded sample: about 10-30 s of host work)."""
    import oracle
    n = (n1, n1, n1)
    f = inputs.fourier_modes(n, wl["kmax"], wl["amp"], wl["seed"])
    p = oracle.Params(*n)
    t = time.perf_counter()
    oracle.step(f, wl["dt"], p, 1)
    dt = time.perf_counter() - t
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=3 * n[0] * n[1] * n[2] / dt / 1e9, unit="GCUPS", cores=threads,
                kind="oracle",
                sample=f"one RK3 step (3 substeps) of the FP64 oracle on {n1}^3 with the "
                       f"same 8-field Fourier-mode recipe, {dt:.1f} s")


def oracle_sweep(inputs, wl, sizes=(64, 256)):
    """The oracle (one RK3 step, same recipe) at each size with one OpenMP
    thread and with every host thread, plus the host's CPU model: the CPU
    side of the measurement, beside the GPU numbers.  Runs on the host only."""
    import ctypes
    import oracle
    gomp = ctypes.CDLL("libgomp.so.1")
    everyone = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = "unknown"
    if os.path.exists("/proc/cpuinfo"):
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    runs = []
    for n1 in sizes:
        n = (n1, n1, n1)
        f = inputs.fourier_modes(n, wl["kmax"], wl["amp"], wl["seed"])
        p = oracle.Params(*n)
        for threads in sorted({1, everyone}):
            gomp.omp_set_num_threads(threads)
            t = time.perf_counter()
            oracle.step(f, wl["dt"], p, 1)
            dt = time.perf_counter() - t
            runs.append(dict(n=n1, threads=threads, seconds=round(dt, 3),
                             gcups=round(3 * n1 ** 3 / dt / 1e9, 6)))
            print(f"# oracle {n1}^3, {threads} thread(s): {dt:.2f} s", file=sys.stderr, flush=True)
    gomp.omp_set_num_threads(everyone)
    return dict(cpu=model, threads_available=everyone, runs=runs)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-sweep", action="store_true",
                    help="only time the CPU oracle (one thread and every thread, at the "
                         "--oracle-sizes grids) and print one JSON line; needs no GPU")
    ap.add_argument("--oracle-sizes", default="64,256",
                    help="comma list of grid sizes n (n^3) for --oracle-sweep")
    ap.add_argument("--precisions", default=None,
                    help="comma list of f64, f32c, f32 (default: f64,f32c; f32c for "
                         "the large workload)")
    ap.add_argument("--workload", default="prec512",
                    choices=["prec512", "sub256", "w0_512", "large1024x512x512"])
    ap.add_argument("--no-segmented", action="store_true",
                    help="skip the timing of the segmented (inner/outer, packed halo "
                         "exchange) step")
    ap.add_argument("--no-order-study", action="store_true",
                    help="skip the timing of stencil orders 2, 4, 6 and 8 at 256^3")
    ap.add_argument("--kernel", default=None, choices=["split", "tiled", "direct"],
                    help="fused-substep kernel (default: the library's default for each "
                         "precision: split for f64, tiled otherwise)")
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed regions of --steps steps per precision (the first is "
                         "the reported one; the median is reported beside it)")
    ap.add_argument("--no-bandwidth", action="store_true",
                    help="skip the copy/triad measurement of achievable HBM bandwidth")
    args = ap.parse_args()
    if args.precisions is None:
        args.precisions = "f32c" if args.workload == "large1024x512x512" else "f64,f32c"
    if args.gpus != 1:
        print("bench.py: this path is one GPU's share of the domain and has no multi-GPU "
              "mode; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.oracle_sweep:
        from paper_2103_01597_amd import inputs
        wl = inputs.WORKLOADS[args.workload]
        sizes = tuple(int(v) for v in args.oracle_sizes.split(","))
        print(json.dumps({"oracle_sweep": oracle_sweep(inputs, wl, sizes),
                          "recipe": f"the {args.workload} field recipe (8 fields, {wl['amp']:g} x "
                                    f"Fourier modes |k|<={wl['kmax']}, seed {wl['seed']}, "
                                    f"dt {wl['dt']:g}) at "
                                    + ", ".join(f"{v}^3" for v in sizes)}))
        return

    import torch
    from paper_2103_01597_amd import inputs, mhd
    mhd.lib()
    torch.cuda.set_device(0)
    wl = inputs.WORKLOADS[args.workload]
    bw = None
    if not args.no_bandwidth:
        bw = achievable_bandwidth(mhd, torch)
        print(f"# bandwidth: {json.dumps(bw)}", file=sys.stderr, flush=True)
    results = {}
    for prec in args.precisions.split(","):
        results[prec] = run_precision(mhd, inputs, torch, args.workload, prec, args.steps,
                                      args.warmup, args.kernel, not args.no_segmented,
                                      max(1, args.repeats))
        print(f"# {prec}: {json.dumps(results[prec])}", file=sys.stderr, flush=True)

    main_prec = "f64" if "f64" in results else next(iter(results))
    r = results[main_prec]
    line = {
        "metric": "GCUPS per RK3 substep at 512^3 (FP64; FP32-storage compensated beside it)"
                  if args.workload == "prec512" else f"GCUPS per RK3 substep ({args.workload})",
        "value": round(r["gcups"], 4),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "ns_per_cell_step": round(r["ms_per_step"] * 1e6 / math.prod(wl["shape"]), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload], "grid": list(wl["shape"]),
                   "precision": main_prec, "kernel": r["kernel"]},
        "roofline": {"bound": "hbm", "achieved": round(r["kernel_gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(r["kernel_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(r["kernel"], main_prec, args.workload),
                     "kernel": KERNEL_SYMBOL[r["kernel"]],
                     "kernel_ms_avg": round(r["kernel_ms_avg"], 4)},
        "ms_per_step_repeats": r["ms_per_step_repeats"],
        "median_gcups": round(r["median_gcups"], 4),
    }
    if bw is not None:
        line["roofline"]["achievable"] = bw["best_gbs"]
        line["roofline"]["frac_of_achievable"] = round(r["kernel_gbs"] / bw["best_gbs"], 4)
        line["bandwidth"] = bw
    for prec, rr in results.items():
        if prec != main_prec:
            line[f"{prec}_gcups"] = round(rr["gcups"], 4)
            line[f"{prec}_roofline_frac"] = round(rr["kernel_gbs"] / HBM_PEAK_GBS, 4)
            line[f"{prec}_kernel_ms_avg"] = round(rr["kernel_ms_avg"], 4)
            line[f"{prec}_kernel"] = KERNEL_SYMBOL[rr["kernel"]]
            line[f"{prec}_traffic"] = measured_traffic(rr["kernel"], prec, args.workload)
            line[f"{prec}_median_gcups"] = round(rr["median_gcups"], 4)
            if bw is not None:
                line[f"{prec}_frac_of_achievable"] = round(rr["kernel_gbs"] / bw["best_gbs"], 4)
    segs = {prec: rr["segmented"] for prec, rr in results.items() if rr["segmented"]}
    if segs:
        line["segmented"] = segs
    if not args.no_order_study:
        line["order_study"] = order_study(mhd, inputs, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(inputs, inputs.WORKLOADS["prec512"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""End-to-end learned-closure run: fine runs of the method -> 4x filtered
training pairs -> training on the GPU -> held-out comparison against the
plain coarse run, with timings.  Prints one JSON line.

    python -m paper_2103_01597_amd.closure_run [--n-fine 256] [--runs 40]
        [--pairs 50] [--epochs 5] [--eval-steps 100]

The 2000 training pairs come from 40 seeded fine runs of 50 pairs each:
more independent initial states (each with its own random wave vectors)
generalise better to the held-out run than fewer, longer runs (measured:
with 10 runs of 200 pairs the corrected run was worse than the plain one
on A_y over the run, with 40 runs of 50 better on every field).
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _timed(torch, fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def conv_throughput(torch, nn, nc, batch):
    """TFLOP/s of the network forward and of forward+backward on random data."""
    net = nn.Closure(seed=1)
    cells = batch * nc ** 3
    x = torch.randn(cells * 8, device="cuda").to(torch.bfloat16)
    y, cache = net.forward(x, nc, batch)
    dy = torch.randn(cells * 8, device="cuda").to(torch.bfloat16)
    ws = torch.empty(nn.wgrad_workspace_floats(nc, batch), device="cuda")
    fwd_ms = _timed(torch, lambda: net.forward(x, nc, batch), 5)
    bwd_ms = _timed(torch, lambda: net.backward(cache, dy, nc, batch, workspace=ws), 5)
    macs = 27 * (8 * 32 + 32 * 32 + 32 * 8)           # per cell, forward
    fwd_flop = 2.0 * macs * cells
    bwd_flop = 2.0 * (macs + 27 * (32 * 8 + 32 * 32)) * cells  # wgrad x3 + dgrad x2
    return dict(fwd_ms=fwd_ms, bwd_ms=bwd_ms, fwd_tflops=fwd_flop / fwd_ms / 1e9,
                bwd_tflops=bwd_flop / bwd_ms / 1e9)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-fine", type=int, default=256)
    ap.add_argument("--runs", type=int, default=40)
    ap.add_argument("--pairs", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=5)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-steps", type=int, default=100)
    ap.add_argument("--kmax", type=int, default=8)
    ap.add_argument("--u-amp", type=float, default=0.1)
    ap.add_argument("--fine-prec", default="f64")
    ap.add_argument("--conv-only", action="store_true",
                    help="only time the network's forward and backward at the coarse size "
                         "(batch --batch) and print that JSON line")
    args = ap.parse_args()

    import torch
    from . import closure, mhd, nn
    if args.conv_only:
        nn.lib()
        print(json.dumps(conv_throughput(torch, nn, args.n_fine // 4, args.batch)), flush=True)
        return
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    amp = (0.0, args.u_amp, args.u_amp, args.u_amp, 0.0, 1e-2, 1e-2, 1e-2)
    nc = args.n_fine // 4
    out = dict(n_fine=args.n_fine, n_coarse=nc, runs=args.runs, pairs=args.runs * args.pairs,
               u_amp=args.u_amp, kmax=args.kmax, fine_prec=args.fine_prec)

    t = time.perf_counter()
    X, D, _ = closure.generate_pairs(n_fine=args.n_fine, runs=args.runs,
                                     pairs_per_run=args.pairs, kmax=args.kmax, amp=amp,
                                     fine_prec=args.fine_prec, log=log)
    out["datagen_s"] = time.perf_counter() - t

    t = time.perf_counter()
    trained, hist = closure.train(X, D, nc, epochs=args.epochs, batch=args.batch, lr=args.lr,
                                  log=log)
    torch.cuda.synchronize()
    out["train_s"] = time.perf_counter() - t
    out["loss_history"] = hist
    del X, D
    torch.cuda.empty_cache()

    ep, ec, truth, plain, corr, truth_dev, fallbacks = closure.evaluate(
        trained, n_fine=args.n_fine, seed=9000, steps=args.eval_steps, kmax=args.kmax, amp=amp,
        fine_prec=args.fine_prec, return_truth=True)
    out["fallbacks"] = fallbacks
    names = mhd.FIELD_NAMES
    for frac in (0.25, 0.5, 1.0):
        i = max(0, int(round(frac * args.eval_steps)) - 1)
        out[f"rel_l2_step{i + 1}"] = {
            "plain": {nm: float(ep[i, q]) for q, nm in enumerate(names)},
            "corrected": {nm: float(ec[i, q]) for q, nm in enumerate(names)}}
    out["mean_rel_l2_u"] = {"plain": float(ep[:, 1:4].mean()), "corrected": float(ec[:, 1:4].mean())}
    out["run_mean_rel_l2"] = {"plain": {nm: float(ep[:, q].mean()) for q, nm in enumerate(names)},
                              "corrected": {nm: float(ec[:, q].mean()) for q, nm in enumerate(names)}}
    out["worst_step_ratio_corrected_over_plain"] = {
        nm: float(np.max(ec[:, q] / ep[:, q])) for q, nm in enumerate(names)}
    ek_t, em_t = closure.shell_spectra(truth)
    ek_p, em_p = closure.shell_spectra(plain)
    ek_c, em_c = closure.shell_spectra(corr)
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))  # noqa: E731
    out["spectrum_rel_err"] = {"kinetic": {"plain": rel(ek_p, ek_t), "corrected": rel(ek_c, ek_t)},
                               "magnetic": {"plain": rel(em_p, em_t), "corrected": rel(em_c, em_t)}}

    # wall time per unit simulated time (dt_fine = 1e-3, coarse dt = 4e-3)
    def step_rate(n, prec, dt, nsteps):
        S = mhd.Solver(n, n, n, prec)
        f = [S.zeros(), S.zeros()]
        f[0].uniform_(0, 1e-2)
        w = S.zeros()
        comp = S.zeros() if prec != "f64" else None
        ms = _timed(torch, lambda: S.step(f, 0, w, comp, dt, nsteps), 2)
        S.close()
        return ms / 1e3 / (nsteps * dt)

    def coarse_rate(tr, nsteps):
        """The coarse run itself, timed end to end with events on the launch
        stream from the held-out filtered state: every coarse step, and for
        the corrected run the copy of the previous state, pack, forward and
        guarded apply."""
        run = closure.CoarseRun(nc, tr)
        run.reset(truth_dev[0])
        dt_c = 4 * 1e-3
        for _ in range(2):
            run.step(dt_c)
        ms = _timed(torch, lambda: run.step(dt_c), nsteps)
        run.close()
        return ms / 1e3 / dt_c

    out["wall_s_per_unit_time"] = {
        f"fine{args.n_fine}_f64": step_rate(args.n_fine, "f64", 1e-3, 20),
        f"fine{args.n_fine}_f32c": step_rate(args.n_fine, "f32c", 1e-3, 20),
        f"coarse{nc}_f32c_plain": coarse_rate(None, 100),
        f"coarse{nc}_f32c_corrected": coarse_rate(trained, 100),
    }
    inf = conv_throughput(torch, nn, nc, 1)
    out["closure_inference_ms_per_step"] = inf["fwd_ms"]
    out["conv_throughput_batch4"] = conv_throughput(torch, nn, nc, 4)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

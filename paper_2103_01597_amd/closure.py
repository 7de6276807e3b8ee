"""Learned closure for a coarse run of the method: data generation, training
and evaluation, driving the library's kernels through the C ABI.

Recipe (the network and data are this library's own; the paper names ML
reconstruction of turbulent flow only as related work, Section 6):

* truth: fine runs of the method (n_f^3, FP64 or FP32C, dt_f) from seeded
  Fourier-mode states; every `ratio` fine steps the state is 4x
  box-filtered to the coarse grid n_c = n_f / 4 (``mhdnn_box_filter4``).
* coarse method: the same solver on n_c^3 in FP32C with dt_c = ratio * dt_f
  (same CFL number since h_c = 4 h_f and ratio = 4).
* pair i: S_i = Step_c(C_i) (one coarse step from the filtered state);
  input T_i = S_i - C_i (the coarse step's tendency), target
  D_i = C_{i+1} - S_i (what the coarse step misses).  The tendency rather
  than the state is the input because the per-step correction is about 1e-4
  of the state, far below BF16's resolution of the state itself, while it
  is a resolvable fraction of the tendency.
* network: periodic conv 8->32->32->8 (``paper_2103_01597_amd.nn.Closure``)
  on the normalised tendency; its output y (per field, in units of the
  target's standard deviation) is added after every coarse step:
  f <- Step_c(f) + y * std_D (``mhdnn_apply``, compensated).
* judged against the plain coarse run by the relative L2 error to the
  filtered truth and by shell spectra of kinetic and magnetic energy.
The plain method stays the fallback: in ``CoarseRun`` a step whose corrected
state would not be finite keeps the plain step's state (a device-side guard
in ``mhdnn_apply``).
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs, mhd, nn


def _solver(n, prec, lengths=None):
    kw = {} if lengths is None else dict(lengths=lengths)
    return mhd.Solver(n, n, n, prec, **kw)


def _to_coarse_solver(S, coarse_flat, buf):
    """Copy an unpadded FP32 [8][n][n][n] tensor into a solver buffer (+halo)."""
    n = S.n[0]
    S.interior_view(buf).copy_(coarse_flat.view(8, n, n, n))
    S.halo_periodic(buf)


def generate_pairs(n_fine=256, runs=40, pairs_per_run=50, seed_base=5000, kmax=8,
                   amp=(0.0, 0.1, 0.1, 0.1, 0.0, 1e-2, 1e-2, 1e-2), dt_fine=1e-3, ratio=4,
                   fine_prec="f64", log=None):
    """Returns (X, D, C0s): coarse-step tendencies and targets, FP32
    [P, 8, n_c^3], and each run's first filtered state."""
    import torch
    nc = n_fine // 4
    F = _solver(n_fine, fine_prec)
    Sc = _solver(nc, "f32c")
    fb = [F.empty(), F.empty()]
    wf = F.zeros()
    compf = F.zeros() if fine_prec == "f32c" else None
    cb = [Sc.empty(), Sc.empty()]
    wc, compc = Sc.zeros(), Sc.zeros()
    P = runs * pairs_per_run
    X = torch.empty((P, 8, nc ** 3), device="cuda")
    D = torch.empty_like(X)
    C0s = []
    snap = torch.empty((pairs_per_run + 1, 8 * nc ** 3), device="cuda")
    k = 0
    for r in range(runs):
        f0 = inputs.fourier_modes((n_fine,) * 3, kmax, amp, seed_base + r)
        F.upload(f0, fb[0])
        cur = 0
        if compf is not None:
            compf.zero_()
        for i in range(pairs_per_run + 1):
            nn.box_filter4(F, fb[cur], snap[i])
            if i < pairs_per_run:
                cur = F.step(fb, cur, wf, compf, dt_fine, ratio)
        C0s.append(snap[0].clone())
        for i in range(pairs_per_run):
            _to_coarse_solver(Sc, snap[i], cb[0])
            compc.zero_()
            c = Sc.step(cb, 0, wc, compc, ratio * dt_fine, 1)
            nn.pair(Sc, cb[c], snap[i], snap[i + 1], X[k], D[k])
            k += 1
        if log:
            log(f"run {r}: {pairs_per_run} pairs")
    torch.cuda.synchronize()
    F.close()
    Sc.close()
    return X, D, C0s


class Trained:
    """A network with its input normalisation and target scale."""

    def __init__(self, net, mean, inv_std, dscale, nc):
        self.net, self.mean, self.inv_std, self.dscale, self.nc = net, mean, inv_std, dscale, nc


def train(X, D, nc, epochs=5, batch=4, lr=2e-3, seed=0, log=None):
    """Fit the closure on (X, D); returns (Trained, per-epoch mean losses)."""
    import torch
    P = X.shape[0]
    cells = nc ** 3
    mean, std = nn.field_stats(X, P, cells)
    std = np.where(std > 0, std, 1.0)
    _, dstd = nn.field_stats(D, P, cells)
    dstd = np.where(dstd > 0, dstd, 1.0)
    inv_std = 1.0 / std
    inv_dstd = 1.0 / dstd
    net = nn.Closure(seed=seed)
    xb = torch.empty(batch * cells * 8, dtype=torch.bfloat16, device="cuda")
    dy = torch.empty(batch * cells * 8, dtype=torch.bfloat16, device="cuda")
    part = torch.empty(256, device="cuda")
    ws = torch.empty(nn.wgrad_workspace_floats(nc, batch), device="cuda")
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(P)
        tot, cnt = 0.0, 0
        for s in range(0, P - batch + 1, batch):
            idx = order[s:s + batch]
            xs = X[idx]  # [batch, 8, cells] (gathered copies)
            ds = D[idx]
            nn.pack(xs, nc, batch, mean, inv_std, xb)
            y, cache = net.forward(xb, nc, batch)
            nn.mse(y, ds, inv_dstd, nc, batch, dy, part)
            grads = net.backward(cache, dy, nc, batch, workspace=ws)
            net.step(grads, lr)
            tot += float(np.sum(part.cpu().numpy(), dtype=np.float64))
            cnt += 1
        hist.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.5f}")
    return Trained(net, mean, inv_std, dstd, nc), hist


def _rel_l2(a, b):
    import torch
    return [float(torch.linalg.vector_norm(a[q] - b[q]) / torch.linalg.vector_norm(b[q]).clamp_min(1e-30))
            for q in range(8)]


class CoarseRun:
    """A coarse FP32C run of the method, plain or with the closure added
    after every step.  The correction is guarded on the device
    (``mhdnn_apply`` with a guard): a step whose corrected state would not be
    finite keeps the plain step's state, with no host round trip; the number
    of such refusals is read once, at the end (``fallbacks``)."""

    def __init__(self, nc, trained=None, lengths=None):
        import torch
        self.S = _solver(nc, "f32c", lengths)
        self.nc, self.trained = nc, trained
        self.cb = [self.S.empty(), self.S.empty()]
        self.w, self.comp = self.S.zeros(), self.S.zeros()
        self.c = 0
        if trained is not None:
            self.prev = self.S.empty()
            self.xb = torch.empty(nc ** 3 * 8, dtype=torch.bfloat16, device="cuda")
            self.guard = torch.zeros(2, dtype=torch.int32, device="cuda")

    def reset(self, coarse_flat):
        _to_coarse_solver(self.S, coarse_flat, self.cb[0])
        self.comp.zero_()
        self.c = 0
        if self.trained is not None:
            self.guard.zero_()

    def step(self, dt):
        """One coarse step (plus the correction); asynchronous."""
        S, t = self.S, self.trained
        if t is not None:
            self.prev.copy_(self.cb[self.c])
        self.c = S.step(self.cb, self.c, self.w, self.comp, dt, 1)
        if t is not None:
            nn.pack_solver(S, self.cb[self.c], t.mean, t.inv_std, self.xb, sub=self.prev)
            y, _ = t.net.forward(self.xb, self.nc, 1)
            nn.apply(S, self.cb[self.c], self.comp, y, t.dscale, guard=self.guard)

    def state(self):
        return self.S.interior_view(self.cb[self.c])

    def fallbacks(self):
        return 0 if self.trained is None else int(self.guard[1].item())

    def close(self):
        self.S.close()


def evaluate(trained, n_fine=256, seed=9000, steps=50, kmax=8,
             amp=(0.0, 0.1, 0.1, 0.1, 0.0, 1e-2, 1e-2, 1e-2), dt_fine=1e-3, ratio=4,
             fine_prec="f64", return_truth=False):
    """Held-out run: filtered fine truth vs plain coarse vs corrected coarse.
    Returns per-step relative L2 errors (plain, corrected) per field and the
    final states (truth, plain, corrected) as host arrays (and, with
    return_truth, the filtered truth of every step on the device)."""
    import torch
    nc = n_fine // 4
    F = _solver(n_fine, fine_prec)
    fb = [F.empty(), F.empty()]
    wf = F.zeros()
    compf = F.zeros() if fine_prec == "f32c" else None
    f0 = inputs.fourier_modes((n_fine,) * 3, kmax, amp, seed)
    F.upload(f0, fb[0])
    truth = torch.empty((steps + 1, 8 * nc ** 3), device="cuda")
    cur = 0
    for i in range(steps + 1):
        nn.box_filter4(F, fb[cur], truth[i])
        if i < steps:
            cur = F.step(fb, cur, wf, compf, dt_fine, ratio)
    F.close()
    del fb, wf
    res = {}
    for mode in ("plain", "corrected"):
        run = CoarseRun(nc, trained if mode == "corrected" else None)
        run.reset(truth[0])
        errs = []
        for i in range(steps):
            run.step(ratio * dt_fine)
            errs.append(_rel_l2(run.state().reshape(8, -1), truth[i + 1].view(8, -1)))
        res[mode] = (np.array(errs), run.state().double().cpu().numpy(), run.fallbacks())
        run.close()
    final_truth = truth[steps].view(8, nc, nc, nc).double().cpu().numpy()
    out = (res["plain"][0], res["corrected"][0], final_truth, res["plain"][1], res["corrected"][1])
    if return_truth:
        return out + (truth, res["corrected"][2])
    return out


def shell_spectra(state, lengths=(2 * math.pi,) * 3):
    """Kinetic (|u|^2/2) and magnetic (|B|^2/2, B = curl A spectrally)
    energy per integer wavenumber shell, from an (8, n, n, n) host state."""
    n = state.shape[-1]
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    shells = np.rint(kmag).astype(int)
    nsh = n // 2 + 1

    def spec(vec):
        e = sum(np.abs(np.fft.fftn(v)) ** 2 for v in vec) / (2 * n ** 6)
        return np.bincount(shells.ravel(), weights=e.ravel(), minlength=nsh)[:nsh]

    u = state[1:4]
    Ah = [np.fft.fftn(a) for a in state[5:8]]
    ik = [1j * KX, 1j * KY, 1j * KZ]
    B = [np.real(np.fft.ifftn(ik[1] * Ah[2] - ik[2] * Ah[1])),
         np.real(np.fft.ifftn(ik[2] * Ah[0] - ik[0] * Ah[2])),
         np.real(np.fft.ifftn(ik[0] * Ah[1] - ik[1] * Ah[0]))]
    return spec(u), spec(B)

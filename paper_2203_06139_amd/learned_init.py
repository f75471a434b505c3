"""Learned fit initialiser: a GELU network trained on plain fits.

The plain method (the baseline): starting point from hf_default_starts, then
fit_batch.  The learned method: rebin each histogram to 256 bins
(hf_rebin_lognorm), predict standardised (m, ln s, ln A, b0, b1) with the
256-512-512-512-5 network (hf_mlp_forward, BF16 MFMA), map back to theta
(hf_target_to_theta), fit_batch from there, and refit every fit that did not
converge from the plain start (fallback).  Training uses the project's own
forward/backward/AdamW step (hf_mlp_train_step) on targets that are the
plain method's fitted parameters.

Everything numeric runs in the library's kernels; torch supplies device
memory, the stream, random initial weights and minibatch index shuffling.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import torch

from . import (FIT_CONVERGED, FP32_BIN, GAUSS_EXP, MLP_HIDDEN, MLP_IN, MLP_OUT, MLP_OUT_PAD,
               POISSON, Model, column_stats, default_starts, fit_batch, mlp_forward, mlp_nparams,
               mlp_train_step, mlp_workspace, rebin_lognorm, target_to_theta, theta_to_target)

MODEL = Model(GAUSS_EXP, 1, -1, 0.0, 1.0)
LAYERS = [(MLP_HIDDEN, MLP_IN), (MLP_HIDDEN, MLP_HIDDEN), (MLP_HIDDEN, MLP_HIDDEN),
          (MLP_OUT_PAD, MLP_HIDDEN)]


def init_params(seed: int, device) -> torch.Tensor:
    """He-normal weights, zero biases; padding rows of the last layer zero."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    parts = []
    for out, inn in LAYERS:
        w = torch.randn(out, inn, generator=g, dtype=torch.float32) * math.sqrt(2.0 / inn)
        if out == MLP_OUT_PAD:
            w *= 0.5
            w[MLP_OUT:] = 0.0
        parts += [w.reshape(-1), torch.zeros(out)]
    p = torch.cat(parts).to(device)
    assert p.numel() == mlp_nparams()
    return p


@dataclass
class FitSet:
    counts: torch.Tensor
    offsets: torch.Tensor
    ranges: torch.Tensor


def plain_fit(fs: FitSet, precision=FP32_BIN, polish_edm=1e-3, edm_tol=1e-10, max_iter=500):
    th0 = default_starts(fs.counts, fs.offsets, fs.ranges, MODEL)
    return th0, fit_batch(fs.counts, fs.offsets, fs.ranges, MODEL, th0, objective=POISSON,
                          precision=precision, polish_edm=polish_edm, edm_tol=edm_tol,
                          max_iter=max_iter)


def physical(res, ranges) -> torch.Tensor:
    """Converged fits whose peak is a peak: mean inside the histogram range,
    width between 0.1% and 50% of it, positive amplitude.  A fit can also
    converge with the Gaussian moved off the data (its gradient vanishes
    there); such fits are no target for a start predictor."""
    lo, hi = ranges[:, 0], ranges[:, 1]
    w = hi - lo
    th = res.theta
    s = th[:, 2].abs()
    return ((res.status == FIT_CONVERGED) & (th[:, 0] > 0) & (th[:, 1] >= lo) & (th[:, 1] <= hi)
            & (s >= 1e-3 * w) & (s <= 0.5 * w) & torch.isfinite(th).all(dim=1))


class LearnedInit:
    def __init__(self, device, seed: int = 0, batch: int = 1024):
        self.device = device
        self.batch = batch
        self.params = init_params(seed, device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.ws = mlp_workspace(batch, device)
        self.step = 0
        self.in_mean = 0.0
        self.in_std = 1.0
        self.t_mean = torch.zeros(MLP_OUT, dtype=torch.float32, device=device)
        self.t_std = torch.ones(MLP_OUT, dtype=torch.float32, device=device)

    # -- data ---------------------------------------------------------------
    def build_training_set(self, n_hist: int, seed: int, nbins: int = 4096, chunk: int = 16384,
                           log=print):
        """Generates n_hist histograms, fits each with the plain method and
        keeps (rebinned input, fitted theta) of the converged fits.  Input and
        target standardisation come from the first chunk."""
        import datagen
        xs, ths = [], []
        kept = 0
        for c0 in range(0, n_hist, chunk):
            B = min(chunk, n_hist - c0)
            counts, off, rg, _ = datagen.batch_case_device(seed + c0, B, nbins, self.device)
            fs = FitSet(counts, off.to(self.device), rg.to(self.device))
            _, res = plain_fit(fs)
            ok = physical(res, fs.ranges)
            if c0 == 0:
                raw = rebin_lognorm(fs.counts, fs.offsets)
                m, s = column_stats(raw.reshape(-1, 1))
                self.in_mean, self.in_std = float(m.item()), float(s.item())
                traw = theta_to_target(res.theta[ok], torch.zeros_like(self.t_mean),
                                       torch.ones_like(self.t_std))
                self.t_mean, self.t_std = column_stats(traw)
            x = rebin_lognorm(fs.counts, fs.offsets, self.in_mean, self.in_std)
            xs.append(x[ok])
            ths.append(res.theta[ok])
            kept += int(ok.sum().item())
            log("training set: %d/%d histograms fitted, %d converged" % (c0 + B, n_hist, kept))
        self.x = torch.cat(xs)
        self.t = theta_to_target(torch.cat(ths), self.t_mean, self.t_std)
        return kept

    # -- training -----------------------------------------------------------
    def train(self, epochs: int, lr: float = 1e-3, wd: float = 1e-4, seed: int = 0, log=print):
        n = (self.x.shape[0] // self.batch) * self.batch
        g = torch.Generator(device=self.device).manual_seed(seed)
        history = []
        for ep in range(epochs):
            perm = torch.randperm(self.x.shape[0], generator=g, device=self.device)[:n]
            tot = torch.zeros((), dtype=torch.float64, device=self.device)
            for b0 in range(0, n, self.batch):
                idx = perm[b0:b0 + self.batch]
                xb = self.x.index_select(0, idx)
                tb = self.t.index_select(0, idx)
                self.step += 1
                lr_t = lr * 0.5 * (1 + math.cos(math.pi * min(1.0, ep / max(1, epochs))))
                mlp_train_step(self.params, self.m, self.v, self.step, max(lr_t, lr * 0.02), wd, xb,
                               tb, self.grads, self.loss, self.ws)
                tot += self.loss[0]
            history.append(float(tot.item()) / (n // self.batch))
            log("epoch %d: mean loss %.5f" % (ep, history[-1]))
        return history

    # -- inference ----------------------------------------------------------
    def predict(self, fs: FitSet) -> torch.Tensor:
        x = rebin_lognorm(fs.counts, fs.offsets, self.in_mean, self.in_std)
        B = x.shape[0]
        Bp = (B + 63) // 64 * 64
        if Bp != B:
            x = torch.cat([x, torch.zeros(Bp - B, MLP_IN, dtype=x.dtype, device=x.device)])
        y = mlp_forward(self.params, x)
        return target_to_theta(y[:B].contiguous(), self.t_mean, self.t_std)

    def fit(self, fs: FitSet, precision=FP32_BIN, polish_edm=1e-3, edm_tol=1e-10, max_iter=500):
        """Fit from the learned start; fits that did not converge to a
        physical peak (see physical) are refitted from the plain start, and
        the refit is kept where it converged to a lower NLL.  Iteration and
        evaluation counts add both attempts.  Returns (result, number of
        fallbacks)."""
        th0 = self.predict(fs)
        res = fit_batch(fs.counts, fs.offsets, fs.ranges, MODEL, th0, objective=POISSON,
                        precision=precision, polish_edm=polish_edm, edm_tol=edm_tol,
                        max_iter=max_iter)
        bad = torch.nonzero(~physical(res, fs.ranges)).reshape(-1)
        nbad = int(bad.numel())
        if nbad:
            sub = subset(fs, bad)
            _, rf = plain_fit(sub, precision, polish_edm, edm_tol, max_iter)
            first_ok = res.status[bad] == FIT_CONVERGED
            take = (rf.status == FIT_CONVERGED) & (~first_ok | (rf.nll < res.nll[bad]))
            idx = bad[take]
            res.theta[idx] = rf.theta[take]
            res.nll[idx] = rf.nll[take]
            res.status[idx] = rf.status[take]
            res.iters[bad] = res.iters[bad] + rf.iters
            res.nevals[bad] = res.nevals[bad] + rf.nevals
        return res, nbad


def subset(fs: FitSet, idx: torch.Tensor) -> FitSet:
    """The histograms idx of a batch, copied into a contiguous batch."""
    off = fs.offsets.cpu()
    ii = idx.cpu().tolist()
    pieces = [fs.counts[int(off[i]):int(off[i + 1])] for i in ii]
    lens = torch.tensor([0] + [int(off[i + 1] - off[i]) for i in ii], dtype=torch.int64)
    return FitSet(torch.cat(pieces), torch.cumsum(lens, 0).to(fs.counts.device),
                  fs.ranges[idx.to(fs.ranges.device)])


def timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0

"""Autotuner of fit_batch's launch shape.

Searches the workgroup size (256 or 512 threads) x persistent workgroups per
CU x the LDS count cache (in bins) x the FP32->FP64 polish threshold by
timing fit_batch (HIP events) on a sample of the batch to be fitted (the
whole batch when `sample` is at least its size), keeps the fastest
configuration whose fits agree with the FP64 fit of the same sample
(|dNLL| < 1e-6 where both converge), then on that shape the size below which
every wave fits a histogram of its own (wave_bins: off, 256 .. 2048 bins),
applies the result to the device's contexts, and caches it as JSON keyed by
(GPU arch, CU count, model, objective, precision).
When no configuration agrees, the shape in place before the search is
restored and RuntimeError is raised.  Cache file: $HF_AUTOTUNE_CACHE or
~/.cache/histfit/autotune.json.
"""
from __future__ import annotations

import itertools
import json
import os

import torch

from . import (FP32_BIN, FP64, POISSON, Model, fit_batch, fit_get_tuning, fit_get_wave_bins,
               fit_max_cache_bins, fit_max_wave_bins, fit_set_tuning, fit_set_wave_bins)

BLOCKS = (256, 512)
WG_PER_CU = (1, 2, 4, 8)
POLISH = (1e-2, 1e-3, 1e-4)
WAVE_BINS = (256, 512, 1024, 2048)
# A wave_bins setting is kept only when it beats the best time so far by
# this fraction.  One wave per histogram makes each of those fits slower
# (a wave instead of a workgroup), which a timed batch need not show: on the
# 4096-histogram Gauss + exponential batch, wave_bins 1024 timed within
# noise of off from the default starts, but made the same batch from
# learned starts 17% slower (7.08 vs 6.05 ms).
WAVE_MARGIN = 0.02


def cache_path() -> str:
    return os.environ.get("HF_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "histfit", "autotune.json"))


def key(model: Model, objective: int, precision: int) -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%dCU/kind%d-g%d-d%d/obj%d/prec%d" % (p.gcnArchName.split(":")[0],
                                                  p.multi_processor_count, model.kind,
                                                  model.n_gauss, model.poly_degree, objective,
                                                  precision)


def _time(fn, reps=2):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_fit(counts, offsets, ranges, model: Model, theta0, objective=POISSON, precision=FP32_BIN,
             sample=512, seed=0, use_cache=True, log=None):
    """Tunes on `sample` histograms drawn from the batch and applies the best
    configuration; returns (config dict, all timings)."""
    from .learned_init import FitSet, subset
    k = key(model, objective, precision)
    path = cache_path()
    if use_cache and os.path.exists(path):
        with open(path) as f:
            known = json.load(f)
        if k in known:
            c = known[k]
            fit_set_tuning(c["wg_per_cu"], c["cache_bins"], c.get("block_size", 256))
            fit_set_wave_bins(c.get("wave_bins", 0))
            return c, []
    before = fit_get_tuning()
    before_waves = fit_get_wave_bins()
    fit_set_wave_bins(0)
    B = offsets.numel() - 1
    g = torch.Generator().manual_seed(seed)
    idx = torch.randperm(B, generator=g)[:min(sample, B)].sort().values
    fs = subset(FitSet(counts, offsets.to(counts.device), ranges.to(counts.device)), idx.to(counts.device))
    th0 = theta0.to(counts.device)[idx.to(counts.device)].contiguous()
    ref = fit_batch(fs.counts, fs.offsets, fs.ranges, model, th0, objective=objective, precision=FP64)
    polishes = POLISH if precision == FP32_BIN else (0.0,)
    space = []
    for blk in BLOCKS:
        cap = max(0, fit_max_cache_bins(model, objective, blk))
        caches = sorted({0, min(cap, 8192), min(cap, 16384), cap})
        space += [(blk, wg, cb, pol) for wg, cb, pol in itertools.product(WG_PER_CU, caches, polishes)]
    results = []
    for blk, wg, cb, pol in space:
        fit_set_tuning(wg, cb, blk)
        run = lambda: fit_batch(fs.counts, fs.offsets, fs.ranges, model, th0, objective=objective,
                                precision=precision, polish_edm=pol)
        ms = _time(run)
        out = run()
        both = (out.status == 0) & (ref.status == 0)
        agree = bool(((out.nll - ref.nll).abs()[both] < 1e-6).all().item())
        results.append(dict(block_size=blk, wg_per_cu=wg, cache_bins=cb, polish_edm=pol, ms=ms,
                            agree=agree))
        if log:
            log(results[-1])
    ok = [r for r in results if r["agree"]]
    if not ok:
        fit_set_tuning(*before)
        fit_set_wave_bins(before_waves)
        raise RuntimeError("no launch shape reproduced the FP64 fits of the sample within 1e-6; "
                           "the previous shape %r is kept" % (before,))
    best = dict(min(ok, key=lambda r: r["ms"]), wave_bins=0)
    fit_set_tuning(best["wg_per_cu"], best["cache_bins"], best["block_size"])
    # second stage, on the chosen shape: one wave per histogram below wave_bins
    capw = fit_max_wave_bins(model, objective, best["block_size"])
    run = lambda: fit_batch(fs.counts, fs.offsets, fs.ranges, model, th0, objective=objective,
                            precision=precision, polish_edm=best["polish_edm"])
    for wb in WAVE_BINS:
        if wb > capw:
            continue
        fit_set_wave_bins(wb)
        ms = _time(run)
        out = run()
        both = (out.status == 0) & (ref.status == 0)
        agree = bool(((out.nll - ref.nll).abs()[both] < 1e-6).all().item())
        r = dict(best, wave_bins=wb, ms=ms, agree=agree)
        results.append(r)
        if log:
            log(r)
        if agree and ms < best["ms"] * (1.0 - WAVE_MARGIN):
            best = r
    fit_set_wave_bins(best["wave_bins"])
    if use_cache:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        known = {}
        if os.path.exists(path):
            with open(path) as f:
                known = json.load(f)
        known[k] = best
        with open(path, "w") as f:
            json.dump(known, f, indent=1)
    return best, results

"""Host-only check of the autotuner's selection rule: a launch shape is only
eligible when its fits reproduce the FP64 fits of the sample, and a search in
which no shape does raises and leaves the previous shape in place.  The
library calls are replaced by stand-ins, so no GPU is needed."""
import pytest
import torch

import paper_2203_06139_amd as hf
from paper_2203_06139_amd import autotune


class _Res:
    def __init__(self, nll):
        B = nll.numel()
        self.nll = nll
        self.status = torch.zeros(B, dtype=torch.int32)
        self.theta = torch.zeros(B, 5, dtype=torch.float64)


def _install(monkeypatch, agreeing, wave_gain=0.0, bad_waves=()):
    """Stand-ins: shapes whose (block, wg) pair is in `agreeing` reproduce the
    FP64 NLLs; every other shape is off by 1e-3, and so is every wave_bins
    in bad_waves.  The time of a shape is its wg_per_cu, less wave_gain per
    1000 wave_bins."""
    state = {"shape": (2, 0, 256), "set": [], "waves": 0}

    def set_tuning(wg, cb, blk=256, device=None):
        state["shape"] = (wg, cb, blk)
        state["set"].append((wg, cb, blk))

    def set_waves(wb, device=None):
        state["waves"] = wb

    def fit_batch(counts, off, rg, model, th0, objective=2, precision=0, polish_edm=0.0, **kw):
        B = off.numel() - 1
        nll = torch.arange(B, dtype=torch.float64)
        wg, _, blk = state["shape"]
        if precision != hf.FP64 and ((blk, wg) not in agreeing or state["waves"] in bad_waves):
            nll = nll + 1e-3
        return _Res(nll)

    monkeypatch.setattr(autotune, "fit_batch", fit_batch)
    monkeypatch.setattr(autotune, "fit_set_tuning", set_tuning)
    monkeypatch.setattr(autotune, "fit_get_tuning", lambda device=None: state["shape"])
    monkeypatch.setattr(autotune, "fit_max_cache_bins", lambda *a, **k: 16384)
    monkeypatch.setattr(autotune, "key", lambda *a: "k")
    monkeypatch.setattr(autotune, "fit_set_wave_bins", set_waves)
    monkeypatch.setattr(autotune, "fit_get_wave_bins", lambda device=None: state["waves"])
    monkeypatch.setattr(autotune, "fit_max_wave_bins", lambda *a, **k: 1500)
    monkeypatch.setattr(autotune, "_time",
                        lambda fn, reps=2: float(state["shape"][0]) - wave_gain * state["waves"] / 1000)
    return state


def _batch(B=8, n=16):
    counts = torch.ones(B * n, dtype=torch.int32)
    off = torch.arange(0, B * n + 1, n, dtype=torch.int64)
    rg = torch.tensor([[0.0, 1.0]] * B, dtype=torch.float64)
    th0 = torch.zeros(B, 5, dtype=torch.float64)
    return counts, off, rg, th0


def test_fastest_agreeing_shape_is_applied(monkeypatch):
    state = _install(monkeypatch, agreeing={(512, 4), (256, 8)})
    best, results = autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3],
                                      sample=8, use_cache=False)
    # the stand-in timing is wg_per_cu, so the fastest agreeing shape is wg 4
    assert (best["block_size"], best["wg_per_cu"]) == (512, 4)
    assert state["shape"][0] == 4 and state["shape"][2] == 512
    assert any(not r["agree"] for r in results)


def test_no_agreeing_shape_raises_and_restores(monkeypatch):
    state = _install(monkeypatch, agreeing=set())
    state["shape"] = (3, 123, 256)
    state["waves"] = 512
    with pytest.raises(RuntimeError, match="no launch shape"):
        autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3], sample=8,
                          use_cache=False)
    assert state["shape"] == (3, 123, 256)
    assert state["waves"] == 512


def test_wave_stage_keeps_the_fastest_agreeing_size(monkeypatch):
    """The second stage tries wave_bins on the chosen shape, within the
    model's limit (1500 here: 2048 is skipped), and keeps the fastest size
    whose fits agree (1024 agrees and is faster than off; 512 ... would be
    slower than 1024)."""
    state = _install(monkeypatch, agreeing={(256, 1)}, wave_gain=0.5, bad_waves=())
    best, results = autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3],
                                      sample=8, use_cache=False)
    assert best["wave_bins"] == 1024 and state["waves"] == 1024
    assert all(r.get("wave_bins", 0) != 2048 for r in results)


def test_wave_stage_skips_disagreeing_sizes(monkeypatch):
    state = _install(monkeypatch, agreeing={(256, 1)}, wave_gain=0.5, bad_waves=(1024,))
    best, _ = autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3], sample=8,
                                use_cache=False)
    assert best["wave_bins"] == 512 and state["waves"] == 512
    state = _install(monkeypatch, agreeing={(256, 1)}, wave_gain=0.0)
    best, _ = autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3], sample=8,
                                use_cache=False)
    assert best["wave_bins"] == 0 and state["waves"] == 0


def test_wave_stage_needs_a_clear_gain(monkeypatch):
    """A wave_bins setting within the margin of the best time (here at most
    0.5% faster) is not taken: one wave per histogram slows each of those
    fits, so only a clear gain on the timed batch counts."""
    state = _install(monkeypatch, agreeing={(256, 1)}, wave_gain=0.005)
    best, results = autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3],
                                      sample=8, use_cache=False)
    assert any(r.get("wave_bins", 0) == 1024 and r["ms"] < 1.0 for r in results)
    assert best["wave_bins"] == 0 and state["waves"] == 0

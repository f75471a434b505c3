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


def _install(monkeypatch, agreeing):
    """Stand-ins: shapes whose (block, wg) pair is in `agreeing` reproduce the
    FP64 NLLs; every other shape is off by 1e-3."""
    state = {"shape": (2, 0, 256), "set": []}

    def set_tuning(wg, cb, blk=256, device=None):
        state["shape"] = (wg, cb, blk)
        state["set"].append((wg, cb, blk))

    def fit_batch(counts, off, rg, model, th0, objective=2, precision=0, polish_edm=0.0, **kw):
        B = off.numel() - 1
        nll = torch.arange(B, dtype=torch.float64)
        wg, _, blk = state["shape"]
        if precision != hf.FP64 and (blk, wg) not in agreeing:
            nll = nll + 1e-3
        return _Res(nll)

    monkeypatch.setattr(autotune, "fit_batch", fit_batch)
    monkeypatch.setattr(autotune, "fit_set_tuning", set_tuning)
    monkeypatch.setattr(autotune, "fit_get_tuning", lambda device=None: state["shape"])
    monkeypatch.setattr(autotune, "fit_max_cache_bins", lambda *a, **k: 16384)
    monkeypatch.setattr(autotune, "key", lambda *a: "k")
    monkeypatch.setattr(autotune, "_time", lambda fn, reps=2: float(state["shape"][0]))
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
    with pytest.raises(RuntimeError, match="no launch shape"):
        autotune.tune_fit(*_batch()[:3], hf.Model(hf.GAUSS_EXP, 1), _batch()[3], sample=8,
                          use_cache=False)
    assert state["shape"] == (3, 123, 256)

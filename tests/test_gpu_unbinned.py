"""GPU parity of nll_unbinned (extended unbinned NLL + gradient) against the
FP64 oracle, with the condition scales the oracle returns:
  |L - L_ref|          <= 1e-10 S_0,  S_0 = |Lambda| + sum |w ln lambda|
  |g_k - g_ref_k|      <= 1e-10 S_k,  S_k = |dLambda_k| + sum |w dlambda_k / lambda|
Sizes cover n = 0, odd tails of the vector path, several blocks, events
outside the range and NaN events, a misaligned (scalar) path, weights, and
the 1e7-event workload in full.
"""
import math

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = [
    (datagen.model_spec(1, 1, 1, 0.0, 5.0), [300.0, 4.0, 0.8, 20.0, 3.0]),
    (datagen.model_spec(1, 2, 3, 5.0, 5.0),
     [200.0, 2.5, 0.5, 150.0, 6.5, 1.1, 30.0, -4.0, 2.0, 0.5]),
    (datagen.model_spec(1, 0, 2, 0.0, 5.0), [40.0, 5.0, 3.0]),
    (datagen.model_spec(1, 1, -1, 0.0, 1.0), [500.0, 5.2, 1.4]),
    (datagen.model_spec(1, 3, 0, 0.0, 1.0), [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 15.0]),
    (datagen.model_spec(1, 4, 3, 5.0, 5.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 50.0, 8.8, 0.3, 15.0, 1.0, -0.5, 0.2]),
    (datagen.model_spec(2, 1, -1, 5.0, 5.0), [300.0, 4.0, 0.8, math.log(20.0), 1.2]),
    (datagen.model_spec(2, 0, -1, 0.0, 5.0), [math.log(80.0), -1.5]),
]


def orc_model(orc, spec):
    return orc.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"])


def gpu_unbinned(hf, spec, x_t, lo, hi, theta, weights=None, want_grad=True):
    import torch
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    nll, g = hf.nll_unbinned(x_t, lo, hi, hf.Model.from_spec(spec), theta, weights=weights,
                             want_grad=want_grad, status=st)
    torch.cuda.synchronize()
    return nll.item(), (None if g is None else g.cpu().numpy()), int(st.item())


def assert_close(ref, nll, grad, what=""):
    assert abs(nll - ref.nll) <= TOL * ref.scales[0], (what, nll, ref.nll)
    if grad is not None:
        err = np.abs(grad - ref.grad)
        assert np.all(err <= TOL * ref.scales[1:]), (what, err / ref.scales[1:])


@pytest.mark.parametrize("case", range(len(CASES)))
def test_unbinned_parity(hf, orc, case):
    import torch
    spec, th = CASES[case]
    lo, hi = 0.0, 10.0
    for n, weighted in ((0, False), (1, True), (2, False), (3, True), (1001, False),
                        (65537, True), (1_000_000, False)):
        x = datagen.unbinned_events(spec, th, lo, hi, n, seed=100 + n + case) if n else np.zeros(0)
        if n > 10:
            # a few events outside the range, and NaN positions: skipped by both
            x[::97] = np.where(np.arange(x[::97].size) % 3 == 0, -1.0,
                               np.where(np.arange(x[::97].size) % 3 == 1, 10.5, math.nan))
        w = (np.random.default_rng(n).uniform(0.5, 1.5, n).astype(np.float32)
             if weighted else None)
        rng = np.random.default_rng(case + n)
        th_eval = np.array(th) * (1 + 0.02 * rng.standard_normal(len(th)))
        ref = orc.unbinned(orc_model(orc, spec), x, lo, hi, th_eval,
                           weights=None if w is None else w.astype(np.float64))
        xt = torch.tensor(x, dtype=torch.float64, device="cuda")
        wt = None if w is None else torch.tensor(w, device="cuda")
        nll, grad, st = gpu_unbinned(hf, spec, xt, lo, hi, th_eval, weights=wt)
        assert st == ref.status
        assert_close(ref, nll, grad, (n, weighted))
        nll_v, _, _ = gpu_unbinned(hf, spec, xt, lo, hi, th_eval, weights=wt, want_grad=False)
        assert abs(nll_v - ref.nll) <= TOL * ref.scales[0]


def test_unbinned_misaligned_and_status(hf, orc):
    import torch
    spec, th = CASES[0]
    x = datagen.unbinned_events(spec, th, 0.0, 10.0, 5001, seed=3)
    xt = torch.tensor(np.concatenate([[0.0], x]), device="cuda")[1:]
    assert xt.data_ptr() % 16 == 8
    ref = orc.unbinned(orc_model(orc, spec), x, 0.0, 10.0, th)
    nll, grad, st = gpu_unbinned(hf, spec, xt, 0.0, 10.0, th)
    assert st == 0
    assert_close(ref, nll, grad, "misaligned")
    xa = torch.tensor(x, device="cuda")
    bad = [300.0, 4.0, 0.8, -20.0, 0.0]  # lambda < 0 in the tails
    nll, grad, st = gpu_unbinned(hf, spec, xa, 0.0, 10.0, bad)
    assert st & 1 and nll == math.inf and np.all(np.isnan(grad))
    nll, grad, st = gpu_unbinned(hf, spec, xa, 0.0, 10.0, [math.nan] + th[1:])
    assert st & 2 and math.isnan(nll) and np.all(np.isnan(grad))
    with pytest.raises(hf.HistfitError):
        hf.nll_unbinned(xa, 1.0, 1.0, hf.Model.from_spec(spec), th)
    with pytest.raises((ValueError, hf.HistfitError)):
        hf.nll_unbinned(xa, 0.0, 1.0, hf.Model(hf.GAUSS2D), [1.0, 0.5, 0.5, 0.1, 0.1, 0.0, 1.0])


def test_unbinned_deterministic(hf):
    import torch
    spec, th = CASES[1]
    x = torch.tensor(datagen.unbinned_events(spec, th, 0.0, 10.0, 200_001, seed=9), device="cuda")
    outs = [gpu_unbinned(hf, spec, x, 0.0, 10.0, th) for _ in range(5)]
    for o in outs[1:]:
        assert o[0] == outs[0][0] and np.array_equal(o[1], outs[0][1])


@pytest.mark.slow
def test_unbinned_full_size_1e7_events(hf, orc):
    """The 1e7-event workload (two Gaussians + cubic on [0, 100]) in full."""
    import torch
    c = datagen.unbinned_case()
    ref = orc.unbinned(orc_model(orc, c["spec"]), c["events"], 0.0, 100.0, c["theta_eval"])
    xt = torch.tensor(c["events"], device="cuda")
    nll, grad, st = gpu_unbinned(hf, c["spec"], xt, 0.0, 100.0, c["theta_eval"])
    assert st == 0
    assert_close(ref, nll, grad, "1e7")

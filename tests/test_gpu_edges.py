"""GPU parity of nll_eval / nll_grad on 1D histograms with bins of any widths
(explicit edges), centre and bin-average models, against the FP64 oracle:
|dNLL| <= 1e-10 S_0, |dgrad_k| <= 1e-10 S_k (the oracle's condition scales)."""
import math

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = [
    (datagen.model_spec(1, 1, 1, 0.0, 1.0), [300.0, 4.8, 0.7, 20.0, -1.2], (0.0, 10.0)),
    (datagen.model_spec(1, 2, 3, 5.0, 5.0),
     [700.0, 3.0, 0.4, 400.0, 6.2, 0.6, 100.0, -20.0, 10.0, 5.0], (0.0, 10.0)),
    (datagen.model_spec(2, 1, -1, 0.0, 1.0), [500.0, 0.45, 0.05, math.log(200.0), math.log(0.3)],
     (0.0, 1.0)),
    (datagen.model_spec(1, 4, 2, 5.0, 5.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 50.0, 8.8, 0.3, 15.0, 1.0, -0.5],
     (0.0, 10.0)),
    (datagen.model_spec(1, 0, 2, 0.5, 2.0), [50.0, 10.0, -8.0], (-2.0, 2.0)),
]


def edges_for(lo, hi, nb, seed):
    w = np.exp(np.random.default_rng(seed).uniform(np.log(0.01), np.log(1.0), nb))
    e = np.concatenate([[0.0], np.cumsum(w)])
    return lo + (hi - lo) * e / e[-1]


def orc_model(orc, spec, avg=0):
    return orc.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"], bin_average=avg)


def counts_for(orc, spec, e, th, avg, seed):
    mu = orc.nll_grad_edges(orc_model(orc, spec, avg), 2, np.zeros(e.size - 1), e, th,
                            want_ell=True).ell
    return np.random.default_rng(seed).poisson(np.maximum(mu, 0.0)).astype(np.uint32)


def gpu(hf, spec, counts, e, theta, obj, avg=0, weights=None, want_grad_w=False):
    import torch
    h = hf.make_hist(counts, (0.0, 1.0), weights=weights, edges=e)
    sp = dict(spec, bin_average=avg)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    nll, grad, gw = hf.nll_grad(h, hf.Model.from_spec(sp), theta, objective=obj,
                                want_grad_w=want_grad_w, status=st)
    ev = hf.nll_eval(h, hf.Model.from_spec(sp), theta, objective=obj)
    torch.cuda.synchronize()
    return (nll.item(), grad.cpu().numpy(), None if gw is None else gw.cpu().numpy(),
            int(st.item()), ev.item())


def check(ref, nll, grad, what):
    assert abs(nll - ref.nll) <= TOL * ref.scales[0], (what, nll, ref.nll)
    err = np.abs(grad - ref.grad)
    assert np.all(err <= TOL * ref.scales[1:]), (what, err / ref.scales[1:])


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_edges_parity(hf, orc, case, obj):
    spec, th, r = CASES[case]
    avgs = (0, 1)
    for avg in avgs:
        for nb, weighted in ((1, False), (3, True), (65, False), (4099, True), (100_003, False)):
            e = edges_for(r[0], r[1], nb, seed=nb + case)
            th_eval = np.array(th) * (1 + 0.02 * np.random.default_rng(nb).standard_normal(len(th)))
            counts = counts_for(orc, spec, e, th, avg, seed=nb + 7)
            w = (np.random.default_rng(nb).uniform(0.5, 1.5, nb).astype(np.float32)
                 if weighted else None)
            ref = orc.nll_grad_edges(orc_model(orc, spec, avg), obj, counts, e, th_eval,
                                     weights=None if w is None else w.astype(np.float64),
                                     want_ell=True)
            nll, grad, gw, st, ev = gpu(hf, spec, counts, e, th_eval, obj, avg, weights=w,
                                        want_grad_w=True)
            assert st == ref.status
            check(ref, nll, grad, (avg, nb, weighted))
            assert ev == nll
            tol = 2e-7 * np.abs(ref.ell) + 1e-11 * (counts.astype(np.float64) + 1.0)
            assert np.all(np.abs(gw.astype(np.float64) - ref.ell) <= tol)


def test_uniform_edges_match_the_uniform_path(hf, orc):
    spec, th, r = CASES[1]
    nb = 20011
    c = datagen.random_1d_case(spec, nb, r[0], r[1], th, seed=4)
    e = np.linspace(r[0], r[1], nb + 1)
    for avg in (0, 1):
        a = gpu(hf, spec, c["counts"], e, c["theta_eval"], 2, avg)
        import torch
        h = hf.make_hist(c["counts"], r)
        nll, grad, _ = hf.nll_grad(h, hf.Model.from_spec(dict(spec, bin_average=avg)),
                                   c["theta_eval"])
        torch.cuda.synchronize()
        ref = orc.nll_grad(orc_model(orc, spec, avg), 2, c["counts"], c["theta_eval"], r)
        assert abs(a[0] - nll.item()) <= 2e-10 * ref.scales[0]
        assert np.all(np.abs(a[1] - grad.cpu().numpy()) <= 2e-10 * ref.scales[1:])


def test_edges_unsupported_calls(hf):
    import torch
    spec, th, r = CASES[0]
    e = edges_for(r[0], r[1], 64, seed=1)
    h = hf.make_hist(np.ones(64, dtype=np.uint32), r, edges=e)
    with pytest.raises(hf.HistfitError):
        hf.nll_grad(h, hf.Model.from_spec(spec), th, precision=hf.FP32_BIN)
    with pytest.raises(hf.HistfitError):
        hf.nll_fisher(h, hf.Model.from_spec(spec), th)
    with pytest.raises(ValueError):
        hf.make_hist(np.ones((4, 4), dtype=np.uint32), r, edges=np.linspace(0, 1, 5))
    with pytest.raises(ValueError):
        hf.make_hist(np.ones(64, dtype=np.uint32), r, edges=e[:-1])
    del torch


@pytest.mark.slow
def test_edges_1e7_bins(hf, orc):
    """1e7 bins of varying widths on [0, 100] with the two-Gaussian + cubic
    model, Poisson, in full."""
    c = datagen.large_fit_case()
    spec = c["spec"]
    e = edges_for(0.0, 100.0, c["nbins"], seed=8)
    ref = orc.nll_grad_edges(orc_model(orc, spec), 2, c["counts"], e, c["theta_eval"], nthreads=8)
    nll, grad, _, st, _ = gpu(hf, spec, c["counts"], e, c["theta_eval"], 2)
    assert st == ref.status
    check(ref, nll, grad, "1e7")

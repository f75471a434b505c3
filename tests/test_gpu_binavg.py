"""GPU parity of the bin-average model (mu_i = the model's average over bin
i) in nll_eval / nll_grad against the FP64 oracle, with the oracle's
condition scales: |dNLL| <= 1e-10 S_0, |dgrad_k| <= 1e-10 S_k."""
import math

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES = [
    (datagen.model_spec(1, 1, 1, 0.0, 1.0), [300.0, 4.8, 0.7, 20.0, -1.2], (0.0, 10.0)),
    (datagen.model_spec(1, 2, 3, 50.0, 50.0),
     [700.0, 30.0, 4.0, 400.0, 62.0, 6.0, 100.0, -20.0, 10.0, 5.0], (0.0, 100.0)),
    (datagen.model_spec(1, 3, 0, 0.0, 1.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 15.0], (0.0, 10.0)),
    (datagen.model_spec(1, 4, 2, 5.0, 5.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 50.0, 8.8, 0.3, 15.0, 1.0, -0.5],
     (0.0, 10.0)),
    (datagen.model_spec(1, 0, 2, 0.5, 2.0), [50.0, 10.0, -8.0], (-2.0, 2.0)),
    (datagen.model_spec(1, 1, -1, 0.0, 1.0), [400.0, 5.0, 1.5], (0.0, 10.0)),
    (datagen.model_spec(2, 1, -1, 0.0, 1.0), [500.0, 0.45, 0.05, math.log(200.0), math.log(0.3)],
     (0.0, 1.0)),
    (datagen.model_spec(2, 2, -1, 5.0, 5.0),
     [300.0, 3.0, 0.4, 200.0, 7.0, 0.7, math.log(30.0), 0.0], (0.0, 10.0)),
]


def avg_spec(spec):
    s = dict(spec)
    s["bin_average"] = 1
    return s


def orc_model(orc, spec):
    return orc.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"], bin_average=1)


def gpu(hf, spec, counts, theta, r, obj, weights=None, want_grad_w=False):
    import torch
    h = hf.make_hist(counts, r, weights=weights)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    nll, grad, gw = hf.nll_grad(h, hf.Model.from_spec(avg_spec(spec)), theta, objective=obj,
                                want_grad_w=want_grad_w, status=st)
    ev = hf.nll_eval(h, hf.Model.from_spec(avg_spec(spec)), theta, objective=obj)
    torch.cuda.synchronize()
    return (nll.item(), grad.cpu().numpy(), None if gw is None else gw.cpu().numpy(),
            int(st.item()), ev.item())


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_bin_average_parity(hf, orc, case, obj):
    spec, th, r = CASES[case]
    for nbins, weighted in ((1, False), (3, True), (65, False), (4099, True), (262147, False)):
        c = datagen.random_1d_case(spec, nbins, r[0], r[1], th, seed=3000 + nbins + case)
        counts = c["counts"]
        if nbins > 10:
            counts[::11] = 0
        w = (np.random.default_rng(nbins).uniform(0.5, 1.5, nbins).astype(np.float32)
             if weighted else None)
        ref = orc.nll_grad(orc_model(orc, spec), obj, counts, c["theta_eval"], r,
                           weights=None if w is None else w.astype(np.float64), want_ell=True)
        nll, grad, gw, st, ev = gpu(hf, spec, counts, c["theta_eval"], r, obj, weights=w,
                                    want_grad_w=True)
        assert st == ref.status
        assert abs(nll - ref.nll) <= TOL * ref.scales[0], (nbins, nll, ref.nll)
        assert ev == nll
        err = np.abs(grad - ref.grad)
        assert np.all(err <= TOL * ref.scales[1:]), (nbins, err / ref.scales[1:])
        # grad_w = l_i per bin in FP32: a rounding of the FP64 term, whose own
        # error is about eps (n + mu) where the Poisson term cancels
        tol = 2e-7 * np.abs(ref.ell) + 1e-11 * (counts.astype(np.float64) + 1.0)
        assert np.all(np.abs(gw.astype(np.float64) - ref.ell) <= tol)


def test_bin_average_differs_from_centre_by_curvature(hf, orc):
    """Sanity against the centre model: for wide bins the two objectives
    differ, and the oracle agrees about by how much."""
    spec, th, r = CASES[5]
    assert spec["kind"] == 1 and spec["poly_degree"] == -1
    c = datagen.random_1d_case(spec, 40, r[0], r[1], th, seed=5)
    nll_avg, _, _, _, _ = gpu(hf, spec, c["counts"], th, r, 2)
    ref_avg = orc.nll_grad(orc_model(orc, spec), 2, c["counts"], th, r).nll
    ref_ctr = orc.nll_grad(orc.Model(1, 1, -1), 2, c["counts"], th, r).nll
    assert abs(ref_avg - ref_ctr) > 1e-3
    assert abs(nll_avg - ref_avg) <= TOL * abs(ref_avg)


def test_bin_average_unsupported_calls(hf):
    import torch
    spec = avg_spec(CASES[0][0])
    m = hf.Model.from_spec(spec)
    h = hf.make_hist(np.ones(64, dtype=np.uint32), (0.0, 10.0))
    with pytest.raises(hf.HistfitError):
        hf.nll_grad(h, m, CASES[0][1], precision=hf.FP32_BIN)
    with pytest.raises(hf.HistfitError):
        hf.nll_fisher(h, m, CASES[0][1])
    c = torch.ones(64, dtype=torch.int32, device="cuda")
    with pytest.raises(hf.HistfitError):
        hf.fit_batch(c, torch.tensor([0, 64], device="cuda"),
                     torch.tensor([[0.0, 10.0]], device="cuda", dtype=torch.float64), m,
                     torch.tensor([CASES[0][1]], device="cuda", dtype=torch.float64))
    bad = hf.Model(hf.GAUSS2D, bin_average=1)
    h2 = hf.make_hist(np.ones((8, 8), dtype=np.uint32), (0.0, 1.0), (0.0, 1.0))
    with pytest.raises((ValueError, hf.HistfitError)):
        hf.nll_grad(h2, bad, [1.0, 0.5, 0.5, 0.1, 0.1, 0.0, 1.0])


@pytest.mark.slow
def test_bin_average_full_size_1e7_bins(hf, orc):
    c = datagen.large_fit_case()
    spec = c["spec"]
    ref = orc.nll_grad(orc_model(orc, spec), 2, c["counts"], c["theta_eval"], c["range"],
                       nthreads=8)
    nll, grad, _, st, _ = gpu(hf, spec, c["counts"], c["theta_eval"], c["range"], 2)
    assert st == 0
    assert abs(nll - ref.nll) <= TOL * ref.scales[0]
    assert np.all(np.abs(grad - ref.grad) <= TOL * ref.scales[1:])

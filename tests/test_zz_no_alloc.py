"""nll_grad_noalloc (the context-free, allocation-free variant of nll_grad)
against nll_grad, through the C ABI, on two calls in a row, the second with a
smaller histogram: the variant keeps its scratch in a device array of the
library shared by every call on the GPU, so the second call must not see the
first call's partials.  Tolerance as for nll_grad against the oracle:
1e-10 of the condition scales S_0, S_k (FP64 bins); in practice the two
entry points run the same kernels over the same grid and agree bit for bit.
"""
import ctypes

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def _call_noalloc(hf, hist, model, theta, obj, seed=None, want_grad_w=False):
    import torch
    dev = hist.counts.device
    th = torch.as_tensor(theta, dtype=torch.float64, device=dev)
    P = th.numel()
    nll = torch.empty(1, dtype=torch.float64, device=dev)
    g = torch.empty(P, dtype=torch.float64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    gw = torch.empty(hist.counts.shape, dtype=torch.float32, device=dev) if want_grad_w else None
    sd = None if seed is None else torch.tensor([seed], dtype=torch.float64, device=dev)
    L = hf.load()
    rc = L.nll_grad_noalloc(ctypes.byref(hist.c()), ctypes.byref(model.c()), obj, hf.FP64,
                            hf._ptr(th), hf._ptr(sd), hf._ptr(nll), hf._ptr(g), hf._ptr(gw), 0,
                            hf._ptr(st), hf._stream(dev))
    assert rc == 0, L.hf_last_error(None)
    return nll, g, gw, st


def test_noalloc_matches_nll_grad_twice_smaller_second(hf, orc):
    import torch
    spec = datagen.model_spec(1, 2, 3, 50.0, 50.0)
    th = [700.0, 30.0, 4.0, 400.0, 62.0, 6.0, 100.0, -20.0, 10.0, 5.0]
    m = hf.Model.from_spec(spec)
    for nbins, obj in ((2_000_003, hf.POISSON), (4099, hf.NEYMAN)):
        c = datagen.random_1d_case(spec, nbins, 0.0, 100.0, th, seed=nbins)
        w = np.random.default_rng(nbins).uniform(0.5, 1.5, nbins).astype(np.float32)
        h = hf.make_hist(c["counts"], (0.0, 100.0), weights=w)
        n1, g1, gw1, s1 = _call_noalloc(hf, h, m, c["theta_eval"], obj, seed=0.75,
                                        want_grad_w=True)
        torch.cuda.synchronize()
        sd = torch.tensor([0.75], dtype=torch.float64, device="cuda")
        n0, g0, gw0 = hf.nll_grad(h, m, c["theta_eval"], objective=obj, seed=sd,
                                  want_grad_w=True)
        torch.cuda.synchronize()
        ref = orc.nll_grad(orc.Model(1, 2, 3, 50.0, 50.0), obj, c["counts"], c["theta_eval"],
                           (0.0, 100.0), weights=w.astype(np.float64))
        assert int(s1.item()) == 0
        assert abs(n1.item() - n0.item()) <= 1e-10 * ref.scales[0], (nbins, n1.item(), n0.item())
        err = np.abs(g1.cpu().numpy() - g0.cpu().numpy())
        assert np.all(err <= 1e-10 * 0.75 * ref.scales[1:]), (nbins, err / ref.scales[1:])
        # against the oracle too (the same bar as nll_grad)
        assert abs(n1.item() - ref.nll) <= 1e-10 * ref.scales[0]
        assert np.all(np.abs(g1.cpu().numpy() - 0.75 * ref.grad) <= 1e-10 * 0.75 * ref.scales[1:])
        np.testing.assert_array_equal(gw1.cpu().numpy(), gw0.cpu().numpy())


def test_noalloc_rejects_bad_arguments(hf):
    import torch
    L = hf.load()
    assert L.nll_grad_noalloc(None, None, 2, 0, None, None, None, None, None, 0, None,
                              None) == -1
    assert b"must not be NULL" in L.hf_last_error(None)
    # an error found by the shared validation is reported the same way
    h = hf.make_hist(np.ones(64, dtype=np.uint32), (1.0, 1.0))
    m = hf.Model(hf.GAUSS_POLY, 1, 1)
    th = torch.zeros(5, dtype=torch.float64, device="cuda")
    out = torch.empty(6, dtype=torch.float64, device="cuda")
    rc = L.nll_grad_noalloc(ctypes.byref(h.c()), ctypes.byref(m.c()), 2, 0, hf._ptr(th), None,
                            hf._ptr(out), hf._ptr(out[1:]), None, 0, None, None)
    assert rc == -1 and b"x range" in L.hf_last_error(None)

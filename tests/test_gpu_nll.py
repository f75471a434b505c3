"""GPU parity of nll_eval / nll_grad against the FP64 CPU oracle.

Tolerances (relative, per the condition scales the oracle returns):
  |NLL_gpu - NLL_ref|       <= tol * S_0,  S_0 = sum |w_i l_i|
  |grad_gpu_k - grad_ref_k| <= tol * S_k,  S_k = sum_i |w_i dl/dmu dmu/dtheta_k|
with tol = 1e-10 for FP64 bins and 1e-5 for FP32-per-bin.  Sizes span one
partial chunk, several blocks and a ragged tail, up to the full 1e7-bin and
2048^2 workloads.
"""
import math

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

TOL = {0: 1e-10, 1: 1e-5}

CASES_1D = [
    (datagen.model_spec(1, 1, 1, 0.0, 1.0), [300.0, 4.8, 0.7, 20.0, -1.2], (0.0, 10.0)),
    (datagen.model_spec(1, 2, 3, 50.0, 50.0),
     [700.0, 30.0, 4.0, 400.0, 62.0, 6.0, 100.0, -20.0, 10.0, 5.0], (0.0, 100.0)),
    (datagen.model_spec(2, 1, -1, 0.0, 1.0), [500.0, 0.45, 0.05, math.log(200.0), math.log(0.3)],
     (0.0, 1.0)),
    (datagen.model_spec(1, 3, 0, 0.0, 1.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 15.0], (0.0, 10.0)),
    (datagen.model_spec(1, 4, 2, 5.0, 5.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 50.0, 8.8, 0.3, 15.0, 1.0, -0.5],
     (0.0, 10.0)),
    (datagen.model_spec(1, 0, 2, 0.5, 2.0), [50.0, 10.0, -8.0], (-2.0, 2.0)),
]


def orc_model(orc, spec):
    return orc.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"])


def gpu_eval(hf, spec, counts, theta, r, obj, prec, weights=None, seed=None, want_grad_w=False):
    import torch
    yr = (r[2], r[3]) if len(r) == 4 else (0.0, 1.0)
    h = hf.make_hist(counts, (r[0], r[1]), yr, weights=weights)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    nll, grad, gw = hf.nll_grad(h, hf.Model.from_spec(spec), theta, objective=obj,
                                precision=prec, seed=seed, want_grad_w=want_grad_w, status=st)
    torch.cuda.synchronize()
    return (nll.item(), grad.cpu().numpy(), None if gw is None else gw.cpu().numpy(),
            int(st.item()))


def assert_close(ref, nll, grad, tol, what="", seed=1.0):
    """grad is seed * dL/dtheta; the NLL is never scaled by the seed."""
    assert abs(nll - ref.nll) <= tol * ref.scales[0], (what, nll, ref.nll, ref.scales[0])
    err = np.abs(grad - seed * ref.grad)
    bound = tol * abs(seed) * ref.scales[1:]
    assert np.all(err <= bound), (what, err / np.maximum(ref.scales[1:], 1e-300))


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES_1D)))
def test_nll_grad_1d_parity(hf, orc, case, obj, prec):
    spec, th, r = CASES_1D[case]
    for nbins, weighted in ((1, False), (3, True), (65, False), (4099, True), (262147, False)):
        c = datagen.random_1d_case(spec, nbins, r[0], r[1], th, seed=1000 + nbins + case)
        counts = c["counts"]
        if nbins > 10:
            counts[::11] = 0
        w = (np.random.default_rng(nbins).uniform(0.5, 1.5, nbins).astype(np.float32)
             if weighted else None)
        ref = orc.nll_grad(orc_model(orc, spec), obj, counts, c["theta_eval"], r,
                           weights=None if w is None else w.astype(np.float64), want_ell=True)
        if weighted:
            # the per-bin weight gradient (grad_w = seed * l_i) on uniform bins,
            # with an upstream seed that also scales the parameter gradient
            import torch
            sd = torch.tensor([0.75], dtype=torch.float64, device="cuda")
            nll, grad, gw, st = gpu_eval(hf, spec, counts, c["theta_eval"], r, obj, prec,
                                         weights=w, seed=sd, want_grad_w=True)
            assert_close(ref, nll, grad, TOL[prec], (nbins, weighted), seed=0.75)
            mu = orc.model_eval(orc_model(orc, spec), c["theta_eval"], (nbins,), r)
            check_grad_w_1d(gw, ref, mu, counts, 0.75, prec)
        else:
            nll, grad, _, st = gpu_eval(hf, spec, counts, c["theta_eval"], r, obj, prec,
                                        weights=w)
            assert_close(ref, nll, grad, TOL[prec], (nbins, weighted))
        assert st == ref.status


def test_fp32_bins_gaussian_only_far_tails(hf, orc):
    """FP32-per-bin with a Gaussian-only model over a range many widths wide:
    in the tails the FP32 exps underflow to 0 (the model is below 1e-38
    there), every tail bin is empty, and the result must still match the
    FP64 oracle within the FP32-per-bin tolerance (Poisson, Neyman) with no
    status bit set."""
    spec = datagen.model_spec(1, 1, -1, 0.0, 1.0)
    r = (0.0, 100.0)
    th = np.array([5e3, 50.0, 1.5])
    for nbins in (4099, 100_003):
        c = datagen.random_1d_case(spec, nbins, r[0], r[1], th, seed=77 + nbins)
        counts = c["counts"]
        x = r[0] + (np.arange(nbins) + 0.5) * (r[1] - r[0]) / nbins
        counts[np.abs(x - th[1]) > 13 * th[2]] = 0
        for obj in (0, 2):
            ref = orc.nll_grad(orc_model(orc, spec), obj, counts, c["theta_eval"], r)
            nll, grad, _, st = gpu_eval(hf, spec, counts, c["theta_eval"], r, obj, 1)
            assert st == 0 and ref.status == 0
            assert np.isfinite(nll) and np.all(np.isfinite(grad))
            assert_close(ref, nll, grad, TOL[1], (nbins, obj))


@pytest.mark.parametrize("prec", [0, 1])
def test_eval_equals_grad_nll_and_is_deterministic(hf, prec):
    import torch
    spec, th, r = CASES_1D[1]
    c = datagen.random_1d_case(spec, 1_000_003, r[0], r[1], th, seed=5)
    h = hf.make_hist(c["counts"], r)
    m = hf.Model.from_spec(spec)
    e = hf.nll_eval(h, m, c["theta_eval"], precision=prec)
    outs = [hf.nll_grad(h, m, c["theta_eval"], precision=prec) for _ in range(10)]
    torch.cuda.synchronize()
    nll0, g0 = outs[0][0].item(), outs[0][1].cpu().numpy()
    assert e.item() == nll0  # same per-bin terms, same reduction tree
    for n, g, _ in outs[1:]:
        assert n.item() == nll0
        assert np.array_equal(g.cpu().numpy(), g0)


@pytest.mark.parametrize("dtype", [np.uint32, np.float32, np.float64])
def test_count_dtypes(hf, orc, dtype):
    spec, th, r = CASES_1D[0]
    c = datagen.random_1d_case(spec, 10_001, r[0], r[1], th, seed=9)
    counts = c["counts"].astype(dtype)
    if dtype != np.uint32:
        counts = counts + np.asarray(0.25, dtype=dtype)  # non-integer counts
    ref = orc.nll_grad(orc_model(orc, spec), 2, counts.astype(np.float64), c["theta_eval"], r)
    nll, grad, _, _ = gpu_eval(hf, spec, counts, c["theta_eval"], r, 2, 0)
    assert_close(ref, nll, grad, 1e-10)


def test_seed_free_mask_and_status(hf, orc):
    import torch
    spec, th, r = CASES_1D[1]
    c = datagen.random_1d_case(spec, 50_000, r[0], r[1], th, seed=3)
    h = hf.make_hist(c["counts"], r)
    m = hf.Model.from_spec(spec)
    seed = torch.tensor([-2.5], dtype=torch.float64, device="cuda")
    nll, g, _ = hf.nll_grad(h, m, c["theta_eval"], seed=seed, free_mask=0b1010010110)
    torch.cuda.synchronize()
    ref = orc.nll_grad(orc_model(orc, spec), 2, c["counts"], c["theta_eval"], r)
    g = g.cpu().numpy()
    mask = np.array([(0b1010010110 >> k) & 1 for k in range(10)], dtype=bool)
    assert np.all(g[~mask] == 0.0)
    assert np.all(np.abs(g[mask] + 2.5 * ref.grad[mask]) <= 2.5e-10 * ref.scales[1:][mask])
    assert abs(nll.item() - ref.nll) <= 1e-10 * ref.scales[0]  # the NLL is not scaled
    # domain error: a negative background makes mu <= 0 in some bins
    bad = np.array(c["theta_eval"])
    bad[6] = -500.0
    refb = orc.nll_grad(orc_model(orc, spec), 2, c["counts"], bad, r)
    nll, grad, _, st = gpu_eval(hf, spec, c["counts"], bad, r, 2, 0)
    assert refb.status & 1 and st & hf.ST_DOMAIN and nll == math.inf
    assert np.all(np.isnan(grad)) and np.all(np.isnan(refb.grad))
    # non-finite theta
    nanth = np.array(c["theta_eval"])
    nanth[1] = math.nan
    nll, grad, _, st = gpu_eval(hf, spec, c["counts"], nanth, r, 2, 0)
    assert st & hf.ST_NONFINITE and not math.isfinite(nll)


def test_host_validation_errors(hf):
    import torch
    spec, th, r = CASES_1D[0]
    m = hf.Model.from_spec(spec)
    counts = torch.ones(17, dtype=torch.int32, device="cuda")
    with pytest.raises(hf.HistfitError):  # misaligned counts pointer
        hf.nll_eval(hf.Hist(counts[1:], r), m, th)
    with pytest.raises(hf.HistfitError):  # wrong range
        hf.nll_eval(hf.Hist(counts, (1.0, 1.0)), m, th)
    with pytest.raises((hf.HistfitError, ValueError)):  # unsupported model
        hf.nll_eval(hf.Hist(counts, r), hf.Model(1, 5, 1), np.zeros(16))
    with pytest.raises(hf.HistfitError):  # bad objective
        hf.nll_eval(hf.Hist(counts, r), m, th, objective=7)


def check_grad_w(orc, gw, ref, th, counts, r, seed, prec):
    """grad_w_i = seed * l_i rounded to FP32.  l_i = mu - n + n ln(n/mu) (or a
    chi-square term) cancels near mu = n, so besides the FP32 output rounding
    the bound allows an absolute error of a few ulps of the operands: FP64
    bins ~1e-14 (mu + n), FP32 hardware transcendentals ~1e-6 |mu - n|."""
    ny, nx = counts.shape
    mu = orc.model_eval(orc.Model(3), th, (ny, nx), r).reshape(-1)
    n = counts.reshape(-1).astype(np.float64)
    expect = seed * ref.ell
    if prec == 0:
        tol = 4e-7 * np.abs(expect) + 1e-14 * abs(seed) * (np.abs(mu) + n)
    else:
        tol = 4e-6 * np.abs(expect) + 2e-6 * abs(seed) * (np.abs(mu - n) + 1e-3 * n)
    err = np.abs(gw.reshape(-1).astype(np.float64) - expect)
    assert np.all(err <= tol + 1e-30), float(np.max(err / (tol + 1e-30)))


def check_grad_w_1d(gw, ref, mu, counts, seed, prec):
    """1D uniform bins: grad_w_i = seed * l_i in FP32, with the same bound as
    the 2D check (the FP32 rounding of the output plus a few ulps of the
    cancelling operands of l)."""
    n = np.asarray(counts, dtype=np.float64).reshape(-1)
    expect = seed * ref.ell
    if prec == 0:
        tol = 4e-7 * np.abs(expect) + 1e-14 * abs(seed) * (np.abs(mu) + n)
    else:
        tol = 4e-6 * np.abs(expect) + 2e-6 * abs(seed) * (np.abs(mu - n) + 1e-3 * n)
    err = np.abs(gw.reshape(-1).astype(np.float64) - expect)
    assert np.all(err <= tol + 1e-30), float(np.max(err / (tol + 1e-30)))


def _case2d(nx, ny, seed):
    rng = np.random.default_rng(seed)
    th = np.array([400.0, 0.45, 0.55, 0.12, 0.09, 0.3, 10.0])
    lam = datagen.intensity_2d(th, nx, ny, (0, 1), (0, 1))
    counts = rng.poisson(lam).astype(np.uint32)
    w = rng.uniform(0.5, 1.5, (ny, nx)).astype(np.float32)
    return counts, w, datagen.perturb(th, 0.02, rng)


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("obj", [0, 1, 2])
def test_nll_grad_2d_parity(hf, orc, obj, prec):
    import torch
    r = (0.0, 1.0, 0.0, 1.0)
    # (64, 64): 16-bin row pieces too wide for the row recurrence (per-bin
    # exps) with vector loads; (513, 257): recurrence, scalar loads, short
    # tail piece per row; (1028, 96): recurrence, vector loads and a 4-bin
    # tail per row, counts as FP64
    for nx, ny in ((1, 1), (37, 29), (64, 64), (513, 257), (1028, 96)):
        counts, w, th = _case2d(nx, ny, nx * 1000 + ny)
        if nx == 1028:
            counts = counts.astype(np.float64)
        ref = orc.nll_grad(orc.Model(3), obj, counts, th, r, weights=w.astype(np.float64),
                           want_ell=True)
        seed = torch.tensor([0.75], dtype=torch.float64, device="cuda")
        nll, grad, gw, st = gpu_eval(hf, datagen.model_spec(3), counts, th, r, obj, prec,
                                     weights=w, seed=seed, want_grad_w=True)
        assert_close(ref, nll, grad, TOL[prec], (nx, ny), seed=0.75)
        check_grad_w(orc, gw, ref, th, counts, r, 0.75, prec)


@pytest.mark.slow
@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("obj", [2, 0])
def test_full_size_1e7_bins(hf, orc, obj, prec):
    """The 1e7-bin two-Gaussian + cubic workload, compared bin-for-bin in full."""
    c = datagen.large_fit_case()
    spec = c["spec"]
    ref = orc.nll_grad(orc_model(orc, spec), obj, c["counts"], c["theta_eval"], c["range"],
                       nthreads=8)
    nll, grad, _, st = gpu_eval(hf, spec, c["counts"], c["theta_eval"], c["range"], obj, prec)
    assert st == 0
    assert_close(ref, nll, grad, TOL[prec])


@pytest.mark.slow
@pytest.mark.parametrize("prec", [0, 1])
def test_full_size_2048_squared(hf, orc, prec):
    import torch
    c = datagen.hist2d_case()
    r = c["range"]
    ref = orc.nll_grad(orc.Model(3), 2, c["counts"], c["theta_eval"], r,
                       weights=c["weights"].astype(np.float64), want_ell=True, nthreads=8)
    nll, grad, gw, st = gpu_eval(hf, c["spec"], c["counts"], c["theta_eval"], r, 2, prec,
                                 weights=c["weights"], want_grad_w=True)
    assert st == 0
    assert_close(ref, nll, grad, TOL[prec])
    check_grad_w(orc, gw, ref, c["theta_eval"], c["counts"], r, 1.0, prec)
    del torch


def test_capture_on_a_stream_never_used_before(hf):
    """A graph captured on a stream the library has not seen (no warm-up call
    on it) takes a spare context, since creating one would allocate during
    capture; replays give the eager result, with eager calls in between."""
    import torch
    spec, th, r = CASES_1D[1]
    c = datagen.random_1d_case(spec, 300_007, r[0], r[1], th, seed=71)
    h = hf.make_hist(c["counts"], r)
    m = hf.Model.from_spec(spec)
    t = torch.as_tensor(c["theta_eval"], dtype=torch.float64, device="cuda")
    n0, g0, _ = hf.nll_grad(h, m, t)
    torch.cuda.synchronize()
    nll = torch.empty(1, dtype=torch.float64, device="cuda")
    grad = torch.empty(10, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            hf.nll_grad(h, m, t, nll_out=nll, grad_out=grad)
    torch.cuda.synchronize()
    for _ in range(3):
        nll.zero_()
        grad.zero_()
        g.replay()
        hf.nll_grad(h, m, t)  # eager work on the default stream between replays
        torch.cuda.synchronize()
        assert torch.equal(nll, n0) and torch.equal(grad, g0)

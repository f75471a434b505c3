"""Pins of the FP64 oracle to things other than itself.

Each check is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign or index, a transposed operand, a wrong constant offset) fails at
least one of them:

* complex-step derivatives (Squire & Trapp 1998) of an independently written
  numpy forward pass, exact to rounding, against the oracle's chain-rule
  gradient;
* 4-point Richardson central differences of the oracle's own NLL;
* product-rule closed forms of the Gaussian chi-square derivatives;
* the zero-gradient invariant at the true parameters on noiseless counts;
* closed-form minimisers of the constant model (mean, harmonic mean, root
  mean square) and the normal equations of a Neyman polynomial fit;
* special points of the model (value A at the mean, A/2 at the half maxima,
  factorisation of the 2D Gaussian at rho = 0);
* Neumaier sums against math.fsum (exactly rounded);
* domain and non-finite handling.
"""
import math

import numpy as np
import pytest

import datagen

POLY1 = dict(kind=1, n_gauss=1, poly_degree=1, t_shift=0.0, t_scale=1.0)


def om(orc, spec):
    return orc.Model(spec["kind"], spec.get("n_gauss", 1), spec.get("poly_degree", -1),
                     spec.get("t_shift", 0.0), spec.get("t_scale", 1.0))


# ---------------------------------------------------------------------------
# An independent numpy forward pass, used only through the complex step.
# ---------------------------------------------------------------------------
def np_mu(spec, th, shape, r):
    if spec["kind"] == 3:
        ny, nx = shape
        x = r[0] + (np.arange(nx) + 0.5) * ((r[1] - r[0]) / nx)
        y = r[2] + (np.arange(ny) + 0.5) * ((r[3] - r[2]) / ny)
        X, Y = np.meshgrid(x, y)
        A, mx, my, sx, sy, rho, c = th
        u = (X - mx) / sx
        v = (Y - my) / sy
        Q = (u * u - 2 * rho * u * v + v * v) / (1 - rho * rho)
        return (A * np.exp(-Q / 2) + c).reshape(-1)
    n = shape[-1]
    x = r[0] + (np.arange(n) + 0.5) * ((r[1] - r[0]) / n)
    mu = np.zeros(n, dtype=np.result_type(th.dtype, np.float64))
    k = 0
    for _ in range(spec["n_gauss"]):
        A, m, s = th[k:k + 3]
        mu = mu + A * np.exp(-((x - m) / s) ** 2 / 2)
        k += 3
    t = (x - spec["t_shift"]) / spec["t_scale"]
    if spec["kind"] == 1:
        for j in range(spec["poly_degree"] + 1):
            mu = mu + th[k + j] * t ** j
    else:
        mu = mu + np.exp(th[k] + th[k + 1] * t)
    return mu


def np_nll(spec, obj, counts, th, r, w=None):
    mu = np_mu(spec, th, counts.shape, r)
    n = counts.reshape(-1).astype(np.float64)
    w = np.ones_like(n) if w is None else w.reshape(-1).astype(np.float64)
    if obj == 0:
        pos = n > 0
        terms = np.where(pos, (n - mu) ** 2 / np.where(pos, n, 1.0), 0.0)
    elif obj == 1:
        terms = (n - mu) ** 2 / mu
    else:
        pos = n > 0
        safe_n = np.where(pos, n, 1.0)
        terms = np.where(pos, mu - n + n * np.log(safe_n / mu), mu)
    return np.sum(w * terms)


def complex_step_grad(spec, obj, counts, th, r, w=None, h=1e-30):
    P = th.size
    g = np.empty(P)
    for k in range(P):
        tc = th.astype(np.complex128)
        tc[k] += 1j * h
        g[k] = np_nll(spec, obj, counts, tc, r, w).imag / h
    return g


CASES_1D = [
    (dict(kind=1, n_gauss=1, poly_degree=1, t_shift=0.0, t_scale=1.0),
     [300.0, 4.8, 0.7, 20.0, -1.2], (0.0, 10.0)),
    (dict(kind=1, n_gauss=2, poly_degree=3, t_shift=50.0, t_scale=50.0),
     [700.0, 30.0, 4.0, 400.0, 62.0, 6.0, 100.0, -20.0, 10.0, 5.0], (0.0, 100.0)),
    (dict(kind=2, n_gauss=1, poly_degree=-1, t_shift=0.0, t_scale=1.0),
     [500.0, 0.45, 0.05, math.log(200.0), math.log(0.3)], (0.0, 1.0)),
    (dict(kind=1, n_gauss=3, poly_degree=0, t_shift=0.0, t_scale=1.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 15.0], (0.0, 10.0)),
]


def _case_counts(spec, th, r, nbins, seed):
    c = datagen.random_1d_case(spec, nbins, r[0], r[1], th, seed, rel=0.03)
    return c["counts"], c["theta_eval"]


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES_1D)))
@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_vs_complex_step_1d(orc, obj, case, weighted):
    spec, th, r = CASES_1D[case]
    counts, th_eval = _case_counts(spec, np.array(th), r, 64, 100 + case)
    counts[::7] = 0  # empty bins exercise the n = 0 branches
    w = np.random.default_rng(7).uniform(0.5, 1.5, counts.size) if weighted else None
    res = orc.nll_grad(om(orc, spec), obj, counts, th_eval, r, weights=w)
    assert res.status == 0
    g_cs = complex_step_grad(spec, obj, counts, th_eval, r, w)
    nll_np = np_nll(spec, obj, counts, th_eval, r, w)
    assert abs(res.nll - nll_np) <= 1e-13 * res.scales[0]
    np.testing.assert_array_less(np.abs(res.grad - g_cs), 1e-12 * res.scales[1:] + 1e-300)


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_vs_complex_step_2d(orc, obj, weighted):
    th = datagen.perturb([400.0, 0.45, 0.55, 0.12, 0.09, 0.3, 10.0], 0.02,
                         np.random.default_rng(3))
    spec = datagen.model_spec(3)
    lam = datagen.intensity_2d(th, 12, 10, (0, 1), (0, 1))
    counts = np.random.default_rng(4).poisson(lam).astype(np.float64)
    counts[0, :3] = 0
    w = np.random.default_rng(5).uniform(0.5, 1.5, counts.shape) if weighted else None
    th_eval = datagen.perturb(th, 0.02, np.random.default_rng(6))
    r = (0.0, 1.0, 0.0, 1.0)
    res = orc.nll_grad(om(orc, spec), obj, counts, th_eval, r, weights=w)
    g_cs = complex_step_grad(spec, obj, counts, th_eval, r, w)
    np.testing.assert_array_less(np.abs(res.grad - g_cs), 1e-12 * res.scales[1:] + 1e-300)


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_gradient_vs_richardson_fd(orc, obj, case):
    spec, th, r = CASES_1D[case]
    counts, th_eval = _case_counts(spec, np.array(th), r, 32, 200 + case)
    M = om(orc, spec)
    res = orc.nll_grad(M, obj, counts, th_eval, r)

    def f(t):
        return orc.nll_grad(M, obj, counts, t, r).nll

    for k in range(th_eval.size):
        h = 1e-4 * max(abs(th_eval[k]), 1e-2)
        e = np.zeros_like(th_eval)
        e[k] = h
        d = (8 * (f(th_eval + e) - f(th_eval - e)) - (f(th_eval + 2 * e) - f(th_eval - 2 * e))) / (12 * h)
        assert abs(d - res.grad[k]) <= 1e-7 * res.scales[1 + k], (k, d, res.grad[k])


def test_gaussian_chi2_product_rule(orc):
    """Neyman chi-square of A exp(-(x-m)^2/2s^2) + b0 + b1 x, derivatives
    written out by the product rule: d chi2/d theta = sum 2 (mu-n)/n dmu/dtheta."""
    spec, th, r = CASES_1D[0]
    counts, th_eval = _case_counts(spec, np.array(th), r, 50, 301)
    counts = counts.astype(np.float64)
    A, m, s, b0, b1 = th_eval
    x = r[0] + (np.arange(50) + 0.5) * (r[1] - r[0]) / 50
    e = np.exp(-(x - m) ** 2 / (2 * s * s))
    mu = A * e + b0 + b1 * x
    pos = counts > 0
    f = np.where(pos, 2 * (mu - counts) / np.where(pos, counts, 1), 0.0)
    expect = np.array([
        np.sum(f * e),
        np.sum(f * A * e * (x - m) / s ** 2),
        np.sum(f * A * e * (x - m) ** 2 / s ** 3),
        np.sum(f),
        np.sum(f * x),
    ])
    res = orc.nll_grad(om(orc, spec), 0, counts, th_eval, r)
    np.testing.assert_allclose(res.grad, expect, rtol=1e-12, atol=1e-12 * res.scales[1:].max())
    assert res.nll == pytest.approx(np.sum(np.where(pos, (counts - mu) ** 2 / np.where(pos, counts, 1), 0)),
                                    rel=1e-13)


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES_1D)))
def test_zero_gradient_at_truth_noiseless(orc, obj, case):
    spec, th, r = CASES_1D[case]
    M = om(orc, spec)
    th = np.array(th)
    n = orc.model_eval(M, th, (200,), r)  # noiseless, real-valued counts
    res = orc.nll_grad(M, obj, n, th, r)
    assert res.nll == 0.0
    assert np.all(res.grad == 0.0)
    off = orc.nll_grad(M, obj, n, th * 1.001, r)
    assert off.nll > 0 and np.linalg.norm(off.grad) > 0


def test_zero_gradient_2d_noiseless(orc):
    M = orc.Model(3)
    th = np.array([500.0, 0.4, 0.6, 0.1, 0.12, -0.35, 7.0])
    r = (0, 1, 0, 1)
    n = orc.model_eval(M, th, (16, 16), r)
    for obj in (0, 1, 2):
        res = orc.nll_grad(M, obj, n, th, r)
        assert res.nll == 0.0 and np.all(res.grad == 0.0)


def _const_model(orc):
    return orc.Model(1, 0, 0)


@pytest.mark.parametrize("weighted", [False, True])
def test_constant_model_closed_form_minimisers(orc, weighted):
    rng = np.random.default_rng(11)
    n = rng.poisson(40.0, 500).astype(np.float64)
    n[:5] = 0
    w = rng.uniform(0.5, 1.5, n.size) if weighted else np.ones(n.size)
    pos = n > 0
    closed = {
        2: np.sum(w * n) / np.sum(w),                    # Poisson: weighted mean
        0: np.sum(w[pos]) / np.sum(w[pos] / n[pos]),     # Neyman: weighted harmonic mean
        1: math.sqrt(np.sum(w * n * n) / np.sum(w)),     # Pearson: weighted RMS
    }
    M = _const_model(orc)
    for obj, c_hat in closed.items():
        res = orc.nll_grad(M, obj, n, [c_hat], (0, 1), weights=w if weighted else None)
        assert abs(res.grad[0]) <= 1e-12 * res.scales[1], obj
        for d in (-0.5, 0.5):
            other = orc.nll_grad(M, obj, n, [c_hat + d], (0, 1), weights=w if weighted else None)
            assert other.nll > res.nll
        fr = orc.fit(M, obj, n, [c_hat * 1.3], (0, 1), weights=w if weighted else None,
                     edm_tol=1e-22)
        assert fr.status == orc.FIT_CONVERGED
        assert fr.theta[0] == pytest.approx(c_hat, rel=1e-8)


def test_neyman_polynomial_normal_equations(orc):
    rng = np.random.default_rng(12)
    nb = 300
    x = (np.arange(nb) + 0.5) * (4.0 / nb) - 2.0
    t = (x - 0.5) / 2.0
    n = rng.poisson(50 + 10 * t - 8 * t * t).astype(np.float64)
    pos = n > 0
    Phi = np.stack([np.ones(nb), t, t * t], axis=1)[pos]
    Wd = 1.0 / n[pos]
    theta_hat = np.linalg.solve(Phi.T @ (Phi * Wd[:, None]), Phi.T @ (Wd * n[pos]))
    M = orc.Model(1, 0, 2, 0.5, 2.0)
    res = orc.nll_grad(M, 0, n, theta_hat, (-2.0, 2.0))
    np.testing.assert_array_less(np.abs(res.grad), 1e-11 * res.scales[1:])
    fr = orc.fit(M, 0, n, theta_hat * np.array([1.1, 0.8, 1.3]), (-2.0, 2.0), edm_tol=1e-22)
    assert fr.status == orc.FIT_CONVERGED
    np.testing.assert_allclose(fr.theta, theta_hat, rtol=1e-7, atol=1e-7)


def test_model_special_points(orc):
    A, m, s = 250.0, 3.0, 0.4
    # a bin centre exactly at m (odd bin count, symmetric range)
    M = orc.Model(1, 1, -1)
    mu = orc.model_eval(M, [A, m, s], (101,), (m - 1.01, m + 1.01))
    assert mu[50] == pytest.approx(A, rel=1e-14)
    # half maxima at m +- s sqrt(2 ln 2): put bin centres there
    hw = s * math.sqrt(2 * math.log(2))
    mu = orc.model_eval(M, [A, m, s], (3,), (m - 1.5 * hw, m + 1.5 * hw))
    np.testing.assert_allclose(mu[[0, 2]], [A / 2, A / 2], rtol=1e-13)
    # polynomial background alone at t = 0 and t = 1
    P = orc.Model(1, 0, 3, 5.0, 2.0)
    mu = orc.model_eval(P, [1.0, 2.0, 3.0, 4.0], (3,), (3.0, 9.0))  # centres 4, 6, 8 -> t = -0.5, 0.5, 1.5
    np.testing.assert_allclose(mu, [1 - 1 + 0.75 - 0.5, 1 + 1 + 0.75 + 0.5, 1 + 3 + 6.75 + 13.5], rtol=1e-14)
    # exponential background
    E = orc.Model(2, 0, -1, 1.0, 1.0)
    mu = orc.model_eval(E, [0.7, -0.3], (2,), (0.0, 4.0))  # centres 1, 3 -> t = 0, 2
    np.testing.assert_allclose(mu, [math.exp(0.7), math.exp(0.7 - 0.6)], rtol=1e-14)
    # 2D: value A + c at the centre; rho = 0 factorises into 1D Gaussians
    M2 = orc.Model(3)
    th2 = [300.0, 0.5, 0.25, 0.1, 0.2, 0.0, 4.0]
    mu2 = orc.model_eval(M2, th2, (9, 11), (0.0, 1.0, -0.2, 0.7))
    gx = orc.model_eval(M, [1.0, 0.5, 0.1], (11,), (0.0, 1.0))
    gy = orc.model_eval(M, [1.0, 0.25, 0.2], (9,), (-0.2, 0.7))
    np.testing.assert_allclose(mu2, 300.0 * np.outer(gy, gx) + 4.0, rtol=1e-13)
    assert mu2[4, 5] == pytest.approx(304.0, rel=1e-14)
    # Q(u=1, v=1) = 2/(1+rho): bin centres at mx+sx, my+sy
    th3 = [1.0, 0.0, 0.0, 1.0, 1.0, 0.4, 0.0]
    mu3 = orc.model_eval(M2, th3, (1, 1), (0.5, 1.5, 0.5, 1.5))
    assert mu3[0, 0] == pytest.approx(math.exp(-1.0 / 1.4), rel=1e-14)


def test_saturated_poisson_offset(orc):
    """sum(mu - n + n ln(n/mu)) - sum(mu - n ln mu) = sum(n ln n - n) for any theta."""
    spec, th, r = CASES_1D[0]
    counts, th_eval = _case_counts(spec, np.array(th), r, 80, 401)
    counts = counts.astype(np.float64)
    M = om(orc, spec)
    mu = orc.model_eval(M, th_eval, (80,), r)
    res = orc.nll_grad(M, 2, counts, th_eval, r)
    pos = counts > 0
    plain = np.sum(mu) - np.sum(counts[pos] * np.log(mu[pos]))
    offset = np.sum(counts[pos] * np.log(counts[pos]) - counts[pos])
    assert res.nll - plain == pytest.approx(offset, rel=1e-12)


def test_neumaier_against_fsum(orc):
    rng = np.random.default_rng(13)
    v = rng.standard_normal(100_000) * np.exp(rng.uniform(-20, 20, 100_000))
    exact = math.fsum(v)
    assert abs(orc.neumaier_sum(v) - exact) <= 2 * np.spacing(abs(exact))
    adv = np.array([1e100, 1.0, -1e100, 1e-3])
    assert orc.neumaier_sum(adv) == math.fsum(adv)
    assert np.sum(adv) != math.fsum(adv)  # naive summation loses it


def test_domain_and_nonfinite(orc):
    M = orc.Model(1, 0, 0)
    n = np.array([3.0, 0.0, 5.0])
    r = (0, 1)
    # Poisson with mu <= 0 and n > 0: +inf, status bit 0
    res = orc.nll_grad(M, 2, n, [-1.0], r)
    assert res.nll == math.inf and res.status & orc.ST_DOMAIN
    assert np.all(np.isnan(res.grad))  # not differentiable at +inf
    # Poisson with mu = 0: the empty bin gives 0, occupied bins are domain errors
    res = orc.nll_grad(M, 2, np.zeros(3), [0.0], r)
    assert res.nll == 0.0 and res.status == 0 and res.grad[0] == 3.0
    # Pearson: mu <= 0 always a domain error
    res = orc.nll_grad(M, 1, n, [0.0], r)
    assert res.nll == math.inf and res.status & orc.ST_DOMAIN
    # Neyman: sign of mu irrelevant, empty bins skipped
    res = orc.nll_grad(M, 0, n, [-1.0], r)
    assert res.nll == pytest.approx(16 / 3 + 36 / 5) and res.status == 0
    # non-finite theta
    res = orc.nll_grad(M, 2, n, [math.nan], r)
    assert res.status & orc.ST_NONFINITE and not math.isfinite(res.nll)


def test_threaded_matches_single(orc):
    c = datagen.single_fit_case()
    M = om(orc, c["spec"])
    a = orc.nll_grad(M, 2, c["counts"], c["theta0"], c["range"])
    b = orc.nll_grad(M, 2, c["counts"], c["theta0"], c["range"], nthreads=5)
    assert b.nll == pytest.approx(a.nll, rel=1e-15)
    np.testing.assert_allclose(b.grad, a.grad, rtol=0, atol=1e-14 * a.scales[1:].max())


def test_fit_recovers_truth_noiseless(orc):
    c = datagen.single_fit_case()
    M = om(orc, c["spec"])
    n = orc.model_eval(M, c["theta_true"], (10_000,), c["range"])
    for obj in (0, 2):
        # the objective is ~0 here with ~1e-8 rounding noise, so EDM 1e-12 is
        # about as far as a decrease can still be verified
        fr = orc.fit(M, obj, n, c["theta0"], c["range"], edm_tol=1e-12, max_iter=1000)
        assert fr.status == orc.FIT_CONVERGED, fr
        np.testing.assert_allclose(fr.theta, c["theta_true"], rtol=1e-5)


def test_fit_end_state_and_hessian(orc):
    c = datagen.single_fit_case()
    M = om(orc, c["spec"])
    fr = orc.fit(M, 2, c["counts"], c["theta0"], c["range"])
    assert fr.status == orc.FIT_CONVERGED
    th = fr.theta
    # fitted values near the generating ones (statistical, seeded)
    np.testing.assert_allclose(th[:3], c["theta_true"][:3], rtol=0.02)
    # the gradient vanishes and the FD Hessian of the NLL is positive definite
    g0 = orc.nll_grad(M, 2, c["counts"], th, c["range"])
    H = np.empty((5, 5))
    for k in range(5):
        h = 1e-5 * max(abs(th[k]), 1e-2)
        e = np.zeros(5)
        e[k] = h
        gp = orc.nll_grad(M, 2, c["counts"], th + e, c["range"]).grad
        gm = orc.nll_grad(M, 2, c["counts"], th - e, c["range"]).grad
        H[:, k] = (gp - gm) / (2 * h)
    H = 0.5 * (H + H.T)
    assert np.all(np.linalg.eigvalsh(H) > 0)
    step = np.linalg.solve(H, g0.grad)
    assert 0.5 * g0.grad @ step < 1e-8  # EDM from the FD Hessian


def test_fit_canonicalises_two_gaussians(orc):
    spec = dict(kind=1, n_gauss=2, poly_degree=0, t_shift=0.0, t_scale=1.0)
    truth = np.array([200.0, 3.0, 0.5, 150.0, 7.0, 0.7, 20.0])
    M = om(orc, spec)
    n = orc.model_eval(M, truth, (400,), (0, 10))
    # start with the Gaussians swapped and one width negative
    start = np.array([160.0, 6.8, -0.6, 190.0, 3.1, 0.45, 18.0])
    fr = orc.fit(M, 2, n, start, (0, 10), edm_tol=1e-12, max_iter=2000)
    assert fr.status == orc.FIT_CONVERGED
    np.testing.assert_allclose(fr.theta, truth, rtol=1e-5)


def test_fig2a_workload_fit(orc):
    """The Fig. 2a fit: gaus started at {100, 1, 3} on 1e5 entries over 1000
    bins of [-5,5] recovers mean 1 and sigma 3 within their statistical errors."""
    c = datagen.fig2a_case()
    M = om(orc, c["spec"])
    fr = orc.fit(M, 2, c["counts"], c["theta0"], c["range"])
    assert fr.status == orc.FIT_CONVERGED
    A, m, s = fr.theta
    assert abs(m - 1.0) < 5 * 0.03 and abs(s - 3.0) < 5 * 0.03
    # the Gaussian's area matches the number of entries inside the range
    phi = lambda z: 0.5 * (1 + math.erf(z / math.sqrt(2)))
    inside = phi((5 - 1) / 3) - phi((-5 - 1) / 3)
    assert A * s * math.sqrt(2 * math.pi) / 0.01 == pytest.approx(c["counts"].sum() / inside, rel=0.02)


# ---------------------------------------------------------------------------
# Expected Hessian (Fisher start of the fitter)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", [0, 1, 2])
def test_fisher_is_the_hessian_at_noiseless_truth(orc, obj, case):
    """Where the counts equal the model, dl/dmu = 0 removes the second
    derivatives of mu from the Hessian, so F must equal it.  The Hessian here
    is a central difference of the complex-step gradient of the independent
    numpy forward pass."""
    spec, th, r = CASES_1D[case]
    M = om(orc, spec)
    th = np.array(th)
    n = orc.model_eval(M, th, (300,), r)
    F = orc.fisher(M, obj, n, th, r)
    H = np.empty_like(F)
    for k in range(th.size):
        h = 1e-4 * max(abs(th[k]), 1e-2)
        e = np.zeros_like(th)
        e[k] = h
        H[:, k] = (complex_step_grad(spec, obj, n, th + e, r) -
                   complex_step_grad(spec, obj, n, th - e, r)) / (2 * h)
    H = 0.5 * (H + H.T)
    d = np.sqrt(np.outer(np.abs(np.diag(H)), np.abs(np.diag(H))))
    assert np.all(np.abs(F - H) <= 1e-5 * d), np.max(np.abs(F - H) / d)


def test_fisher_2d_is_the_hessian_at_noiseless_truth(orc):
    spec = dict(kind=3)
    M = orc.Model(3)
    th = np.array([500.0, 0.4, 0.6, 0.1, 0.12, -0.35, 7.0])
    r = (0, 1, 0, 1)
    n = orc.model_eval(M, th, (24, 24), r)
    for obj in (0, 1, 2):
        F = orc.fisher(M, obj, n, th, r)
        H = np.empty_like(F)
        for k in range(th.size):
            h = 1e-4 * max(abs(th[k]), 1e-2)
            e = np.zeros_like(th)
            e[k] = h
            H[:, k] = (complex_step_grad(spec, obj, n, th + e, r) -
                       complex_step_grad(spec, obj, n, th - e, r)) / (2 * h)
        H = 0.5 * (H + H.T)
        d = np.sqrt(np.outer(np.abs(np.diag(H)), np.abs(np.diag(H))))
        assert np.all(np.abs(F - H) <= 1e-5 * d), (obj, np.max(np.abs(F - H) / d))


def test_fisher_constant_model_closed_form(orc):
    rng = np.random.default_rng(21)
    n = rng.poisson(40.0, 400).astype(np.float64)
    n[:7] = 0
    w = rng.uniform(0.5, 1.5, n.size)
    M = _const_model(orc)
    c = 37.0
    closed = {2: np.sum(w) / c, 1: 2 * np.sum(w) / c, 0: 2 * np.sum(w[n > 0] / n[n > 0])}
    for obj, val in closed.items():
        F = orc.fisher(M, obj, n, [c], (0, 1), weights=w)
        assert F.shape == (1, 1)
        assert F[0, 0] == pytest.approx(val, rel=1e-13), obj


def test_fisher_scoring_step_is_the_poisson_constant_mle(orc):
    """For mu = c the Fisher-scoring step from any c0 > 0 lands on the
    weighted mean: c1 = c0 - g/F = sum(w n)/sum(w).  So the Fisher-started
    fit takes one iteration."""
    rng = np.random.default_rng(22)
    n = rng.poisson(25.0, 300).astype(np.float64)
    w = rng.uniform(0.5, 1.5, n.size)
    M = _const_model(orc)
    c_hat = np.sum(w * n) / np.sum(w)
    for c0 in (3.0, 20.0, 90.0):
        fr = orc.fit(M, 2, n, [c0], (0, 1), weights=w, edm_tol=1e-22, hessian_init=1)
        assert fr.status == orc.FIT_CONVERGED
        assert fr.iters == 1, fr
        assert fr.theta[0] == pytest.approx(c_hat, rel=1e-12)
        plain = orc.fit(M, 2, n, [c0], (0, 1), weights=w, edm_tol=1e-22, hessian_init=0)
        assert plain.theta[0] == pytest.approx(c_hat, rel=1e-8) and plain.iters > fr.iters


def test_fisher_start_cuts_iterations_on_batch(orc):
    """Same fits from the default starts with and without the Fisher start:
    the minima agree and the Fisher start needs far fewer iterations."""
    from oracle import mlp as omlp
    c = datagen.batch_case(seed=31, B=48, lo_bins=256, hi_bins=8192)
    M = orc.Model(2, 1, -1, 0.0, 1.0)
    counts = c["counts"].astype(np.float64)
    th0 = omlp.default_starts(counts, c["offsets"], c["ranges"])
    r0 = orc.fit_many(M, 2, counts, c["offsets"], c["ranges"], th0, nthreads=8, hessian_init=0)
    r1 = orc.fit_many(M, 2, counts, c["offsets"], c["ranges"], th0, nthreads=8, hessian_init=1)
    both = (r0[2] == 0) & (r1[2] == 0)
    assert both.mean() > 0.9
    assert np.median(np.abs(r1[1] - r0[1])[both]) < 1e-6
    assert r1[3].mean() < 0.5 * r0[3].mean(), (r1[3].mean(), r0[3].mean())


# ---------------------------------------------------------------------------
# Parameter covariance from the expected Hessian
# ---------------------------------------------------------------------------
def test_covariance_constant_model_textbook_variances(orc):
    """Poisson counts: the MLE of a constant is the mean, whose variance is
    c/N.  Neyman: the fit is the weighted mean with sigma_i^2 = n_i, whose
    variance is 1/sum(1/n_i).  Pearson: sigma_i^2 = mu, variance c/N."""
    rng = np.random.default_rng(31)
    n = rng.poisson(25.0, 300).astype(np.float64)
    M = _const_model(orc)
    N = n.size
    chat = n.mean()
    cov, ok = orc.covariance(orc.fisher(M, 2, n, [chat], (0, 1)), 2)
    assert ok and cov[0, 0] == pytest.approx(chat / N, rel=1e-12)
    cov, ok = orc.covariance(orc.fisher(M, 1, n, [chat], (0, 1)), 1)
    assert ok and cov[0, 0] == pytest.approx(chat / N, rel=1e-12)
    cov, ok = orc.covariance(orc.fisher(M, 0, n, [chat], (0, 1)), 0)
    assert ok and cov[0, 0] == pytest.approx(1.0 / np.sum(1.0 / n), rel=1e-12)


def test_covariance_neyman_line_is_the_least_squares_covariance(orc):
    """A straight line fitted by Neyman's chi-square is weighted least squares
    with sigma_i^2 = n_i; its covariance is inv(Phi^T W Phi), W = diag(1/n)."""
    rng = np.random.default_rng(32)
    nb = 80
    n = rng.poisson(60.0, nb).astype(np.float64) + 1.0
    r = (0.0, 4.0)
    M = orc.Model(1, 0, 1)
    x = r[0] + (np.arange(nb) + 0.5) * (r[1] - r[0]) / nb
    Phi = np.stack([np.ones(nb), x], axis=1)
    expect = np.linalg.inv(Phi.T @ (Phi / n[:, None]))
    cov, ok = orc.covariance(orc.fisher(M, 0, n, [60.0, 1.0], r), 0)
    assert ok
    np.testing.assert_allclose(cov, expect, rtol=1e-11)


def test_covariance_free_mask_and_singular(orc):
    F = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    cov, ok = orc.covariance(F, 2, free_mask=0b101)
    assert ok
    sub = np.linalg.inv(F[np.ix_([0, 2], [0, 2])])
    assert cov[1, :].tolist() == [0, 0, 0] and cov[:, 1].tolist() == [0, 0, 0]
    np.testing.assert_allclose(cov[np.ix_([0, 2], [0, 2])], sub, rtol=1e-14)
    cov, ok = orc.covariance(np.array([[1.0, 1.0], [1.0, 1.0 - 1e-300]]) - np.eye(2) * 1e-3, 0)
    assert not ok and np.all(np.isnan(cov))


@pytest.mark.parametrize("obj", [0, 2])
def test_covariance_matches_the_spread_of_refits(orc, obj):
    """Monte Carlo: refit many Poisson replicas of one Gaussian on a flat
    background; the sample covariance of the fitted parameters must match
    2 UP inv(F) at the truth (a factor-2 mistake in UP would be off by 100%).
    With 600 replicas a variance is known to sqrt(2/599) = 6%."""
    R, nb = 600, 60
    r = (0.0, 6.0)
    th = np.array([400.0, 3.0, 0.5, 80.0])
    M = orc.Model(1, 1, 0)
    mu = orc.model_eval(M, th, (nb,), r)
    rng = np.random.default_rng(33)
    counts = rng.poisson(np.tile(mu, (R, 1))).astype(np.float64)
    off = np.arange(R + 1, dtype=np.int64) * nb
    ranges = np.tile(np.array(r), (R, 1))
    fits, _, st, _, _ = orc.fit_many(M, obj, counts.reshape(-1), off, ranges, np.tile(th, (R, 1)),
                                     nthreads=8, hessian_init=1)
    assert np.all(st == orc.FIT_CONVERGED)
    emp = np.cov(fits.T)
    cov, ok = orc.covariance(orc.fisher(M, obj, mu, th, r), obj)
    assert ok
    np.testing.assert_allclose(np.diag(emp), np.diag(cov), rtol=0.25)
    corr = lambda C: C[0, 2] / math.sqrt(C[0, 0] * C[2, 2])  # amplitude-width correlation
    assert abs(corr(emp) - corr(cov)) < 0.12

"""Pins of the bin-average model (the model's integral over each bin divided
by the bin width, instead of its value at the centre) in the oracle: the
per-bin averages against adaptive quadrature of an independent numpy
intensity, and the objective's gradient against complex-step derivatives of
a numpy forward pass of the averaged model."""
import math

import numpy as np
import pytest
from scipy import integrate, special

CASES = [
    (1, 1, [300.0, 4.0, 0.8, 20.0, 3.0], (0.0, 10.0), 40),
    (2, 3, [200.0, 2.5, 0.5, 150.0, 6.5, 1.1, 30.0, -4.0, 2.0, 0.5], (0.0, 10.0), 25),
    (1, 0, [500.0, 5.2, 0.05, 2.0], (0.0, 10.0), 64),   # bins wider than the Gaussian
    (0, 3, [40.0, 5.0, 3.0, -1.0], (-3.0, 7.0), 7),
]
T_SHIFT, T_SCALE = 1.0, 5.0


def _model(orc, ng, deg):
    return orc.Model(1, ng, deg, T_SHIFT, T_SCALE, bin_average=1)


def np_f(th, x, ng, deg):
    lam = 0.0 * x
    for g in range(ng):
        A, m, s = th[3 * g: 3 * g + 3]
        lam = lam + A * np.exp(-((x - m) / s) ** 2 / 2)
    t = (x - T_SHIFT) / T_SCALE
    for j in range(deg + 1):
        lam = lam + th[3 * ng + j] * t ** j
    return lam


def np_avg(th, a, b, ng, deg):
    """Averaged model, complex-capable: Gaussian by the complex erf, the
    polynomial by its antiderivative."""
    h = b - a
    mu = 0.0 * a
    for g in range(ng):
        A, m, s = th[3 * g: 3 * g + 3]
        mu = mu + A * s * math.sqrt(math.pi / 2) * (special.erf((b - m) / (s * math.sqrt(2))) -
                                                     special.erf((a - m) / (s * math.sqrt(2)))) / h
    ta, tb = (a - T_SHIFT) / T_SCALE, (b - T_SHIFT) / T_SCALE
    for j in range(deg + 1):
        mu = mu + th[3 * ng + j] * T_SCALE * (tb ** (j + 1) - ta ** (j + 1)) / ((j + 1) * h)
    return mu


@pytest.mark.parametrize("case", range(len(CASES)))
def test_bin_average_by_quadrature(orc, case):
    ng, deg, th, r, nb = CASES[case]
    mu = orc.model_eval(_model(orc, ng, deg), th, (nb,), r)
    h = (r[1] - r[0]) / nb
    for i in range(nb):
        a, b = r[0] + i * h, r[0] + (i + 1) * h
        q, _ = integrate.quad(lambda x: float(np_f(np.array(th), np.array([x]), ng, deg)[0]), a, b,
                              epsabs=0, epsrel=1e-13, limit=200)
        assert mu[i] == pytest.approx(q / h, rel=1e-11, abs=1e-12 * np.max(np.abs(mu))), i


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_gradient_by_complex_step(orc, case, obj):
    ng, deg, th, r, nb = CASES[case]
    M = _model(orc, ng, deg)
    lam = orc.model_eval(M, th, (nb,), r)
    n = np.random.default_rng(case).poisson(np.maximum(lam, 0.5)).astype(np.float64)
    n[::5] = np.maximum(n[::5], 1.0)
    ref = orc.nll_grad(M, obj, n, th, r)
    h_bin = (r[1] - r[0]) / nb
    a = r[0] + np.arange(nb) * h_bin
    b = a + h_bin

    def L(tc):
        mu = np_avg(tc, a + 0j, b + 0j, ng, deg)
        if obj == 0:
            pos = n > 0
            return np.sum(np.where(pos, (n - mu) ** 2 / np.where(pos, n, 1), 0))
        if obj == 1:
            return np.sum((n - mu) ** 2 / mu)
        return np.sum(mu - n + np.where(n > 0, n * np.log(np.where(n > 0, n, 1) / mu), 0))

    assert ref.nll == pytest.approx(float(np.real(L(np.array(th, dtype=complex)))), rel=1e-12)
    hs = 1e-30
    for k in range(len(th)):
        tc = np.array(th, dtype=complex)
        tc[k] += 1j * hs
        cs = np.imag(L(tc)) / hs
        assert abs(ref.grad[k] - cs) <= 1e-11 * ref.scales[1 + k], (k, ref.grad[k], cs)


def test_polynomial_average_closed_form(orc):
    """The averages of t^j used per bin: 1, t_c, t_c^2 + d^2/3, t_c^3 + t_c d^2."""
    for deg in range(4):
        th = [0.0] * deg + [1.0]
        mu = orc.model_eval(orc.Model(1, 0, deg, T_SHIFT, T_SCALE, bin_average=1), th, (5,),
                            (-2.0, 8.0))
        for i in range(5):
            a, b = -2.0 + 2 * i, -2.0 + 2 * (i + 1)
            q, _ = integrate.quad(lambda x: ((x - T_SHIFT) / T_SCALE) ** deg, a, b, epsrel=1e-14)
            assert mu[i] == pytest.approx(q / 2.0, rel=1e-13, abs=1e-15)


# ---------------------------------------------------------------------------
# Bins of any widths (explicit edges)
# ---------------------------------------------------------------------------
def _edges(lo, hi, nb, seed):
    """Ascending edges with widths varying over two orders of magnitude."""
    w = np.exp(np.random.default_rng(seed).uniform(np.log(0.01), np.log(1.0), nb))
    e = np.concatenate([[0.0], np.cumsum(w)])
    return lo + (hi - lo) * e / e[-1]


def _mu_from_ell(orc, M, edges, th):
    # Poisson with n = 0 gives l_i = mu_i exactly
    return orc.nll_grad_edges(M, 2, np.zeros(edges.size - 1), edges, th, want_ell=True).ell


@pytest.mark.parametrize("case", range(len(CASES)))
def test_edges_centre_and_average_values(orc, case):
    ng, deg, th, r, nb = CASES[case]
    e = _edges(r[0], r[1], nb, seed=case)
    centre = orc.Model(1, ng, deg, T_SHIFT, T_SCALE)
    mu_c = _mu_from_ell(orc, centre, e, th)
    mid = 0.5 * (e[:-1] + e[1:])
    np.testing.assert_allclose(mu_c, np_f(np.array(th), mid, ng, deg), rtol=1e-13,
                               atol=1e-13 * np.max(np.abs(mu_c)))
    mu_a = _mu_from_ell(orc, _model(orc, ng, deg), e, th)
    for i in range(nb):
        q, _ = integrate.quad(lambda x: float(np_f(np.array(th), np.array([x]), ng, deg)[0]),
                              e[i], e[i + 1], epsabs=0, epsrel=1e-13, limit=200)
        assert mu_a[i] == pytest.approx(q / (e[i + 1] - e[i]), rel=1e-10,
                                        abs=1e-11 * np.max(np.abs(mu_a))), i


@pytest.mark.parametrize("avg", [0, 1])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_edges_gradient_by_complex_step(orc, case, avg):
    ng, deg, th, r, nb = CASES[case]
    e = _edges(r[0], r[1], nb, seed=10 + case)
    M = orc.Model(1, ng, deg, T_SHIFT, T_SCALE, bin_average=avg)
    mu = _mu_from_ell(orc, M, e, th)
    n = np.random.default_rng(case).poisson(np.maximum(mu, 0.5)).astype(np.float64)
    ref = orc.nll_grad_edges(M, 2, n, e, th)

    def L(tc):
        m = (np_avg(tc, e[:-1] + 0j, e[1:] + 0j, ng, deg) if avg else
             np_f(tc, 0.5 * (e[:-1] + e[1:]) + 0j, ng, deg))
        return np.sum(m - n + np.where(n > 0, n * np.log(np.where(n > 0, n, 1) / m), 0))

    assert ref.nll == pytest.approx(float(np.real(L(np.array(th, dtype=complex)))), rel=1e-12)
    for k in range(len(th)):
        tc = np.array(th, dtype=complex)
        tc[k] += 1j * 1e-30
        cs = np.imag(L(tc)) / 1e-30
        assert abs(ref.grad[k] - cs) <= 1e-11 * ref.scales[1 + k], (k, ref.grad[k], cs)


def test_uniform_edges_reproduce_the_range_form(orc):
    ng, deg, th, r, nb = CASES[1]
    n = np.random.default_rng(2).poisson(30, nb).astype(np.float64)
    e = np.linspace(r[0], r[1], nb + 1)
    for avg in (0, 1):
        M = orc.Model(1, ng, deg, T_SHIFT, T_SCALE, bin_average=avg)
        a = orc.nll_grad_edges(M, 1, n, e, th)
        b = orc.nll_grad(M, 1, n, th, r)
        assert abs(a.nll - b.nll) <= 1e-13 * b.scales[0]
        assert np.all(np.abs(a.grad - b.grad) <= 1e-13 * b.scales[1:])


# ---------------------------------------------------------------------------
# Exponential background: bin average and unbinned integral
# ---------------------------------------------------------------------------
EXP_CASES = [
    (1, [300.0, 4.0, 0.8, math.log(20.0), 0.6]),
    (0, [math.log(50.0), -2.5]),
    (1, [200.0, 6.0, 0.5, math.log(5.0), 0.0]),    # b1 = 0: S(0) = 1, S'(0) = 0
    (2, [100.0, 2.0, 0.4, 80.0, 7.0, 1.0, math.log(3.0), 4.0]),
]


def np_exp_f(th, x, ng):
    lam = 0.0 * x
    for g in range(ng):
        A, m, s = th[3 * g: 3 * g + 3]
        lam = lam + A * np.exp(-((x - m) / s) ** 2 / 2)
    return lam + np.exp(th[3 * ng] + th[3 * ng + 1] * (x - T_SHIFT) / T_SCALE)


def np_exp_avg(th, a, b, ng):
    h = b - a
    mu = 0.0 * a
    for g in range(ng):
        A, m, s = th[3 * g: 3 * g + 3]
        mu = mu + A * s * math.sqrt(math.pi / 2) * (special.erf((b - m) / (s * math.sqrt(2))) -
                                                     special.erf((a - m) / (s * math.sqrt(2)))) / h
    # the average of exp(b0 + b1 t) over [t_c - d, t_c + d] written as
    # exp(b0 + b1 t_c) sinh(u)/u, u = b1 d: exact, and unlike the difference
    # of antiderivatives free of cancellation for small b1 d (the complex
    # step then differentiates it to full accuracy)
    b0, b1 = th[3 * ng], th[3 * ng + 1]
    ta, tb = (a - T_SHIFT) / T_SCALE, (b - T_SHIFT) / T_SCALE
    tc, d = 0.5 * (ta + tb), 0.5 * (tb - ta)
    u = b1 * d
    return mu + np.exp(b0 + b1 * tc) * np.sinh(u) / u


@pytest.mark.parametrize("case", range(len(EXP_CASES)))
def test_exp_bin_average_by_quadrature(orc, case):
    ng, th = EXP_CASES[case]
    e = _edges(0.0, 10.0, 30, seed=40 + case)
    M = orc.Model(2, ng, -1, T_SHIFT, T_SCALE, bin_average=1)
    mu = _mu_from_ell(orc, M, e, th)
    for i in range(e.size - 1):
        q, _ = integrate.quad(lambda x: float(np_exp_f(np.array(th), np.array([x]), ng)[0]),
                              e[i], e[i + 1], epsabs=0, epsrel=1e-13, limit=200)
        assert mu[i] == pytest.approx(q / (e[i + 1] - e[i]), rel=1e-11), i


@pytest.mark.parametrize("case", range(len(EXP_CASES)))
def test_exp_bin_average_gradient_by_complex_step(orc, case):
    ng, th = EXP_CASES[case]
    if th[-1] == 0.0:
        th = th[:-1] + [1e-3]  # the complex step needs b1 != 0 in the antiderivative form
    e = _edges(0.0, 10.0, 40, seed=50 + case)
    M = orc.Model(2, ng, -1, T_SHIFT, T_SCALE, bin_average=1)
    n = np.random.default_rng(case).poisson(np.maximum(_mu_from_ell(orc, M, e, th), 0.5))
    ref = orc.nll_grad_edges(M, 2, n.astype(np.float64), e, th)

    def L(tc):
        m = np_exp_avg(tc, e[:-1] + 0j, e[1:] + 0j, ng)
        return np.sum(m - n + np.where(n > 0, n * np.log(np.where(n > 0, n, 1) / m), 0))

    for k in range(len(th)):
        tc = np.array(th, dtype=complex)
        tc[k] += 1j * 1e-30
        cs = np.imag(L(tc)) / 1e-30
        assert abs(ref.grad[k] - cs) <= 1e-10 * ref.scales[1 + k], (k, ref.grad[k], cs)


@pytest.mark.parametrize("case", range(len(EXP_CASES)))
def test_exp_unbinned_integral_and_gradient(orc, case):
    """Lambda for the exponential background over the whole range, where
    b1 (t_hi - t_lo)/2 reaches the closed-form branch, against quadrature;
    the gradient against the complex step."""
    ng, th = EXP_CASES[case]
    M = orc.Model(2, ng, -1, T_SHIFT, T_SCALE)
    lo, hi = 0.0, 10.0
    r0 = orc.unbinned(M, np.array([]), lo, hi, th)
    q, _ = integrate.quad(lambda x: float(np_exp_f(np.array(th), np.array([x]), ng)[0]), lo, hi,
                          epsabs=0, epsrel=1e-13, limit=200)
    assert r0.nll == pytest.approx(q, rel=1e-12)
    if th[-1] == 0.0:
        th = th[:-1] + [1e-3]
    x = np.random.default_rng(case).uniform(lo, hi, 300)
    r = orc.unbinned(M, x, lo, hi, th)

    def L(tc):
        Lam = 0.0
        for g in range(ng):
            A, m, s = tc[3 * g: 3 * g + 3]
            Lam = Lam + A * s * math.sqrt(math.pi / 2) * (
                special.erf((hi - m) / (s * math.sqrt(2))) - special.erf((lo - m) / (s * math.sqrt(2))))
        b0, b1 = tc[3 * ng], tc[3 * ng + 1]
        tl, th_ = (lo - T_SHIFT) / T_SCALE, (hi - T_SHIFT) / T_SCALE
        u = b1 * 0.5 * (th_ - tl)
        Lam = Lam + (hi - lo) * np.exp(b0 + b1 * 0.5 * (tl + th_)) * np.sinh(u) / u
        return Lam - np.sum(np.log(np_exp_f(tc, x + 0j, ng)))

    for k in range(len(th)):
        tc = np.array(th, dtype=complex)
        tc[k] += 1j * 1e-30
        cs = np.imag(L(tc)) / 1e-30
        assert abs(r.grad[k] - cs) <= 1e-11 * r.scales[1 + k], (k, r.grad[k], cs)

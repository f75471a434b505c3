"""Pins of the extended unbinned NLL oracle (oracle.unbinned): the integral
term against quadrature, the gradient against complex-step derivatives of an
independent numpy forward pass, and textbook maximum-likelihood estimates at
which the gradient must vanish."""
import math

import numpy as np
import pytest
from scipy import integrate, special


def _model(orc, ng, deg):
    return orc.Model(1, ng, deg, 0.0, 5.0)


def np_lambda(th, x, ng, deg, t_scale=5.0):
    lam = 0.0 * x
    for g in range(ng):
        A, m, s = th[3 * g: 3 * g + 3]
        lam = lam + A * np.exp(-((x - m) / s) ** 2 / 2)
    t = x / t_scale
    for j in range(deg + 1):
        lam = lam + th[3 * ng + j] * t ** j
    return lam


def np_L(th, x, lo, hi, ng, deg, w=None):
    """Forward pass with complex support: the Gaussian integral through the
    complex erf, the polynomial's by its antiderivative."""
    w = np.ones(x.size) if w is None else w
    Lam = 0.0
    for g in range(ng):
        A, m, s = th[3 * g: 3 * g + 3]
        Lam = Lam + A * s * math.sqrt(math.pi / 2) * (special.erf((hi - m) / (s * math.sqrt(2))) -
                                                      special.erf((lo - m) / (s * math.sqrt(2))))
    for j in range(deg + 1):
        Lam = Lam + th[3 * ng + j] * 5.0 * ((hi / 5.0) ** (j + 1) - (lo / 5.0) ** (j + 1)) / (j + 1)
    return Lam - np.sum(w * np.log(np_lambda(th, x, ng, deg)))


CASES = [(1, 1, [300.0, 4.0, 0.8, 20.0, 3.0]), (2, 3, [200.0, 2.5, 0.5, 150.0, 6.5, 1.1,
                                                       30.0, -4.0, 2.0, 0.5]),
         (0, 2, [40.0, 5.0, 3.0]), (1, -1, [500.0, 5.2, 1.4])]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_integral_term_by_quadrature(orc, case):
    ng, deg, th = CASES[case]
    lo, hi = 0.0, 10.0
    r = orc.unbinned(_model(orc, ng, deg), np.array([]), lo, hi, th)
    quad, _ = integrate.quad(lambda x: float(np_lambda(np.array(th), np.array([x]), ng, deg)[0]),
                             lo, hi, epsabs=0, epsrel=1e-13, limit=200)
    assert r.nll == pytest.approx(quad, rel=1e-12)


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_gradient_by_complex_step(orc, case, weighted):
    ng, deg, th = CASES[case]
    rng = np.random.default_rng(case)
    x = rng.uniform(0, 10, 400)
    w = rng.uniform(0.5, 1.5, x.size) if weighted else None
    r = orc.unbinned(_model(orc, ng, deg), x, 0.0, 10.0, th, weights=w)
    assert r.status == 0
    assert r.nll == pytest.approx(float(np.real(np_L(np.array(th), x, 0, 10, ng, deg, w))),
                                  rel=1e-13, abs=1e-12 * r.scales[0])
    h = 1e-30
    for k in range(len(th)):
        tc = np.array(th, dtype=complex)
        tc[k] += 1j * h
        ref = np.imag(np_L(tc, x, 0.0, 10.0, ng, deg, w)) / h
        assert abs(r.grad[k] - ref) <= 1e-12 * r.scales[1 + k], (k, r.grad[k], ref)


def test_gaussian_mle_is_stationary(orc):
    """A pure Gaussian intensity on a range 40 widths wide: the maximum
    likelihood estimates are yield A s sqrt(2 pi) = N, m = sample mean,
    s = population standard deviation, where the gradient vanishes."""
    x = np.random.default_rng(3).normal(50.0, 2.0, 5000)
    N = x.size
    m, s = x.mean(), x.std()
    A = N / (s * math.sqrt(2 * math.pi))
    r = orc.unbinned(_model(orc, 1, -1), x, -30.0, 130.0, [A, m, s])
    assert np.all(np.abs(r.grad) <= 1e-10 * r.scales[1:]), r.grad / r.scales[1:]


def test_constant_mle_and_value(orc):
    x = np.random.default_rng(4).uniform(0, 8, 777)
    c = x.size / 8.0
    r = orc.unbinned(_model(orc, 0, 0), x, 0.0, 8.0, [c])
    assert abs(r.grad[0]) <= 1e-12 * r.scales[1]
    assert r.nll == pytest.approx(x.size - x.size * math.log(c), rel=1e-13)


def test_range_weights_and_domain(orc):
    ng, deg, th = CASES[0]
    M = _model(orc, ng, deg)
    x = np.random.default_rng(5).uniform(0, 10, 300)
    base = orc.unbinned(M, x, 0.0, 10.0, th)
    outside = orc.unbinned(M, np.concatenate([x, [-1.0, 10.5, 99.0]]), 0.0, 10.0, th)
    assert outside.nll == base.nll and np.array_equal(outside.grad, base.grad)
    w = np.ones(x.size)
    w[7] = 2.0
    dup = orc.unbinned(M, np.concatenate([x, [x[7]]]), 0.0, 10.0, th)
    wt = orc.unbinned(M, x, 0.0, 10.0, th, weights=w)
    assert wt.nll == pytest.approx(dup.nll, rel=1e-14)
    np.testing.assert_allclose(wt.grad, dup.grad, rtol=1e-12)
    bad = orc.unbinned(M, x, 0.0, 10.0, [300.0, 4.0, 0.8, -20.0, 0.0])  # lambda < 0 in the tails
    assert bad.status & 1 and bad.nll == math.inf and np.all(np.isnan(bad.grad))
    nf = orc.unbinned(M, x, 0.0, 10.0, [math.nan, 4.0, 0.8, 20.0, 3.0])
    assert nf.status & 2 and math.isnan(nf.nll)

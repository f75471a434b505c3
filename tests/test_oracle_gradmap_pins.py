"""Pins of the elementwise Gaussian gradient-map oracle (oracle/gradmap.py),
each against something other than the oracle's own reverse sweep."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import gradmap as og


def _inputs(n=257, seed=3):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-3, 3, n)
    s = rng.uniform(0.3, 2.5, n)
    x = p + s * rng.uniform(-6, 6, n)
    return x, p, s


@pytest.mark.parametrize("norm", [og.NORM_LISTING, og.NORM_PDF])
def test_complex_step_derivatives(norm):
    """d/dx, d/dp, d/dsigma by the complex step on the forward function (exact
    to rounding, independent of the reverse sweep)."""
    x, p, s = _inputs()
    _, xb, pb, sb = og.grad_map(x, p, s, norm)
    h = 1e-30
    a = og.norm_exponent(norm)

    def g_c(xc, pc, sc):
        d = xc - pc
        return (2 * math.pi) ** -0.5 * sc ** -a * np.exp(-d * d / (2 * sc * sc))

    cx = np.imag(g_c(x + 1j * h, p + 0j, s + 0j)) / h
    cp = np.imag(g_c(x + 0j, p + 1j * h, s + 0j)) / h
    cs = np.imag(g_c(x + 0j, p + 0j, s + 1j * h)) / h
    for got, ref in ((xb, cx), (pb, cp), (sb, cs)):
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


def test_listing_derivative_identities():
    """The closed forms the listing's generated gradient must satisfy:
    dg/dx = -g (x - p)/sigma^2 = -dg/dp, checked at 512 elements; at x = p
    both vanish and g is the normalisation itself."""
    rng = np.random.default_rng(4)
    n = 512
    x = rng.normal(0, 2, n)
    p = rng.normal(0, 2, n)
    s = 1.7
    g, xb, pb, _ = og.grad_map(x, p, s)
    np.testing.assert_array_equal(xb, -pb)
    xb2 = np.where(np.isclose(x, p), 0, xb)
    np.testing.assert_allclose(xb2 * s * s / (-(x - p) * g), 1.0, rtol=1e-13)
    g0, xb0, pb0, _ = og.grad_map(p, p, s)
    assert np.all(xb0 == 0) and np.all(pb0 == 0)
    np.testing.assert_allclose(g0, (2 * math.pi) ** -0.5 * s ** -0.5, rtol=1e-15)


@pytest.mark.parametrize("norm,expect", [(og.NORM_LISTING, lambda s: math.sqrt(s)),
                                         (og.NORM_PDF, lambda s: 1.0)])
def test_normalisation_by_quadrature(norm, expect):
    """Integral over x: sigma^(1/2) for the listing's normalisation, 1 for the
    pdf (adaptive quadrature, independent of the formula's constant)."""
    for s in (0.4, 1.0, 3.5):
        val, err = integrate.quad(lambda x: float(og.gauss(np.array([x]), 0.7, s, norm)[0]),
                                  -np.inf, np.inf, epsabs=0, epsrel=1e-12)
        assert val == pytest.approx(expect(s), rel=1e-10)


def test_seed_scales_and_shared_adjoint_is_derivative_of_the_sum():
    """Adjoints are linear in the seed; the adjoint of a shared sigma is
    d/dsigma of sum_i w_i g_i (complex step on the weighted total)."""
    x, p, _ = _inputs(n=300, seed=5)
    s = 1.3
    w = np.random.default_rng(6).uniform(-2, 2, x.size)
    g, xb, pb, sb = og.grad_map(x, p, s, og.NORM_LISTING, seed=w)
    g1, xb1, pb1, sb1 = og.grad_map(x, p, s, og.NORM_LISTING)
    np.testing.assert_array_equal(g, g1)
    np.testing.assert_allclose(xb, w * xb1, rtol=1e-15)
    h = 1e-30
    tot = lambda sc: np.sum(w * (2 * math.pi) ** -0.5 * sc ** -0.5 *
                            np.exp(-(x - p) ** 2 / (2 * sc * sc)))
    ref = np.imag(tot(s + 1j * h)) / h
    assert og.shared_sum(sb) == pytest.approx(ref, rel=1e-12)
    refp = np.imag(np.sum(w * (2 * math.pi) ** -0.5 * s ** -0.5 *
                          np.exp(-(x - (p[0] + 1j * h)) ** 2 / (2 * s * s)))) / h
    _, _, pbs, _ = og.grad_map(x, p[0], s, og.NORM_LISTING, seed=w)
    assert og.shared_sum(pbs) == pytest.approx(refp, rel=1e-12)

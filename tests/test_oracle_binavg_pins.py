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

"""Pins of the learned-initialiser oracle (oracle/mlp.py) to outside facts:
torch's own BF16 round-to-nearest-even cast and AdamW, values of Phi, central
finite differences of the FP64 network, count conservation of the rebinning,
and recovery of a known peak by the default-start heuristic."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp as om


def test_bf16_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * np.exp(rng.uniform(-30, 30, 10000)),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -1.0 - 2 ** -8, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(om.bf16(x), ref)


def test_gelu_values_and_derivative():
    assert om.gelu(np.array([0.0]))[0] == 0.0
    phi1 = 0.5 * (1 + math.erf(1 / math.sqrt(2)))
    assert om.gelu(np.array([1.0]))[0] == pytest.approx(phi1, rel=1e-15)
    assert om.gelu(np.array([-1.0]))[0] == pytest.approx(-(1 - phi1), rel=1e-14)
    z = np.linspace(-5, 5, 101)
    h = 1e-6
    fd = (om.gelu(z + h) - om.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(om.gelu_prime(z), fd, atol=1e-9)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = om.init_params(3)
    x = rng.standard_normal((4, om.IN))
    t = rng.standard_normal((4, om.OUT))
    loss, g, _ = om.loss_and_grad(p, x, t, rounding=False)
    # random coordinates of every layer, and one random direction
    idx = []
    for (wo, bo), (out, inn) in zip(om.OFFSETS, om.LAYERS):
        rows = min(out, om.OUT) if out == om.OUT_PAD else out
        idx += list(wo + rng.integers(0, rows * inn, 6)) + list(bo + rng.integers(0, rows, 2))
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-5
        fd = (om.loss_and_grad(p + e, x, t, False)[0] - om.loss_and_grad(p - e, x, t, False)[0]) / 2e-5
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i
    v = rng.standard_normal(p.size)
    v[om.OFFSETS[3][0] + om.OUT * om.HIDDEN:om.OFFSETS[3][1]] = 0  # padding rows stay zero
    v[om.OFFSETS[3][1] + om.OUT:] = 0
    eps = 1e-6
    fd = (om.loss_and_grad(p + eps * v, x, t, False)[0] - om.loss_and_grad(p - eps * v, x, t, False)[0]) / (2 * eps)
    assert fd == pytest.approx(g @ v, rel=1e-6)
    assert np.all(g[om.OFFSETS[3][0] + om.OUT * om.HIDDEN:om.OFFSETS[3][1]] == 0)


def test_adamw_matches_torch():
    rng = np.random.default_rng(2)
    p0 = rng.standard_normal(50)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.AdamW([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-3)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 5):
        g = rng.standard_normal(50)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = om.adamw_step(p, m, v, g, step, 1e-2, 1e-3)
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("nb", [100, 256, 4096, 5000])
def test_rebin_conserves_counts(nb):
    rng = np.random.default_rng(nb)
    c = rng.poisson(50, nb).astype(np.float64)
    out = om.rebin_lognorm(c, [0, nb], 0.0, 1.0)[0]
    j = ((2 * np.arange(nb) + 1) * 256) // (2 * nb)
    k = np.bincount(j, minlength=256)
    sums = np.where(k > 0, np.expm1(out) * k, 0.0)
    assert sums.sum() == pytest.approx(c.sum(), rel=1e-12)
    if nb % 256 == 0:
        blocks = c.reshape(256, nb // 256).sum(axis=1)
        np.testing.assert_allclose(sums, blocks, rtol=1e-12)


def test_default_starts_recover_a_clean_peak():
    nb = 4096
    x = (np.arange(nb) + 0.5) / nb
    A, m, s, bk = 800.0, 0.37, 0.02, 50.0
    c = np.rint(A * np.exp(-0.5 * ((x - m) / s) ** 2) + bk)
    th = om.default_starts(c, [0, nb], [(0.0, 1.0)])[0]
    assert abs(th[1] - m) <= 2.0 / nb
    assert th[2] == pytest.approx(s, rel=0.1)
    assert th[0] == pytest.approx(A, rel=0.05)
    assert th[3] == pytest.approx(math.log(bk), abs=0.05)
    assert abs(th[4]) < 0.1


def test_target_maps_round_trip():
    rng = np.random.default_rng(4)
    th = np.stack([np.exp(rng.uniform(4, 9, 20)), rng.uniform(0, 1, 20), rng.uniform(0.01, 0.05, 20),
                   rng.uniform(2, 7, 20), rng.uniform(-3, 3, 20)], axis=1)
    mean = rng.standard_normal(5)
    std = rng.uniform(0.5, 2, 5)
    t = om.theta_to_target(th, mean, std)
    y = np.zeros((20, om.OUT_PAD))
    y[:, :5] = t
    np.testing.assert_allclose(om.target_to_theta(y, mean, std), th, rtol=1e-12)
    mu, sd = om.column_stats(t)
    np.testing.assert_allclose(mu, t.mean(axis=0), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(sd, t.std(axis=0), rtol=1e-12)


def test_default_starts_steep_background_has_no_false_edge_peak():
    """Backgrounds rising 20x to 100x across the range with a peak inside:
    against a straight line through the edge means the convex background
    itself leaves the largest excess at the steep edge (x = 0.996 in every
    case below); against the exponential through the edge means the start
    lands on the peak and b1 on the background slope."""
    nb = 16384
    x = (np.arange(nb) + 0.5) / nb
    for A, m, s, rise in ((120, 0.5, 0.02, 46), (60, 0.4, 0.03, 46), (200, 0.3, 0.02, 100),
                          (40, 0.5, 0.02, 20)):
        c = np.rint(A * np.exp(-0.5 * ((x - m) / s) ** 2) + 20.0 * np.exp(math.log(rise) * x))
        th = om.default_starts(c, [0, nb], [(0.0, 1.0)])[0]
        assert abs(th[1] - m) < 0.005, (A, m, s, rise, th)
        assert th[4] == pytest.approx(math.log(rise), rel=0.02), (A, m, s, rise, th)

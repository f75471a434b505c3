"""Seeded synthetic histograms for the histogram-fit workloads.

This module serves both the oracle-side tests and the GPU path, so it holds
none of the method's arithmetic: it never evaluates the bin-centre model, the
fit objective or any derivative.  Counts are drawn as Poisson variates whose
means are the *bin integrals* of the generating intensity divided by the bin
width (exact normal-CDF differences for Gaussians, exact antiderivatives for
polynomial and exponential backgrounds, a 2x2 Gauss-Legendre rule over each
bin for the correlated 2D Gaussian).  That is how a real histogram is filled
(paper, sec. 4, Fig. 2a fills its histogram from the function by sampling),
and it differs from the bin-centre value the method evaluates by O(h^2/s^2).

Every generator takes an explicit seed and uses numpy's PCG64, except
batch_case_device, which draws the same distribution with seeded torch
generators on a device (for training sets of ~1e6 histograms).

Model descriptors are plain dicts {kind, n_gauss, poly_degree, t_shift,
t_scale}; kind 1 = Gaussians + polynomial in t = (x - t_shift)/t_scale,
kind 2 = Gaussians + exp(b0 + b1 t), kind 3 = 2D correlated Gaussian +
constant.  Parameter order: (A, m, s) per Gaussian, then background
coefficients; 2D: (A, mx, my, sx, sy, rho, c).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

GAUSS_POLY, GAUSS_EXP, GAUSS2D = 1, 2, 3


def model_spec(kind, n_gauss=1, poly_degree=-1, t_shift=0.0, t_scale=1.0):
    return dict(kind=kind, n_gauss=n_gauss, poly_degree=poly_degree, t_shift=float(t_shift),
                t_scale=float(t_scale))


def nparams(spec) -> int:
    if spec["kind"] == GAUSS2D:
        return 7
    nb = spec["poly_degree"] + 1 if spec["kind"] == GAUSS_POLY else 2
    return 3 * spec["n_gauss"] + nb


# --------------------------------------------------------------------------
# Bin-integrated intensities (divided by the bin width)
# --------------------------------------------------------------------------
def _edges(lo, hi, n):
    i = np.arange(n + 1, dtype=np.float64)
    return lo + i * ((hi - lo) / n)


def _gauss_bin_mean(A, m, s, a, b):
    """(1/h) * integral_a^b A exp(-((x-m)/s)^2/2) dx via normal-CDF differences.

    Right of the mean the survival function is differenced instead of the CDF
    so that neither side loses digits to 1 - small."""
    za = (a - m) / s
    zb = (b - m) / s
    right = za >= 0
    p = np.where(right, special.ndtr(-za) - special.ndtr(-zb), special.ndtr(zb) - special.ndtr(za))
    return A * s * math.sqrt(2.0 * math.pi) * p / (b - a)


def _poly_bin_mean(c, t_shift, t_scale, a, b):
    ta = (a - t_shift) / t_scale
    tb = (b - t_shift) / t_scale
    tot = np.zeros_like(a)
    for j, cj in enumerate(c):
        tot += cj * (tb ** (j + 1) - ta ** (j + 1)) / (j + 1)
    return tot * t_scale / (b - a)


def _exp_bin_mean(b0, b1, t_shift, t_scale, a, b):
    ta = (a - t_shift) / t_scale
    tb = (b - t_shift) / t_scale
    if b1 == 0.0:
        return np.full_like(a, math.exp(b0))
    return np.exp(b0 + b1 * ta) * np.expm1(b1 * (tb - ta)) / (b1 * (tb - ta))


def intensity_1d(spec, theta, nbins, lo, hi):
    """Bin-integrated mean counts per bin for the 1D generating models."""
    e = _edges(lo, hi, nbins)
    a, b = e[:-1], e[1:]
    lam = np.zeros(nbins, dtype=np.float64)
    k = 0
    for _ in range(spec["n_gauss"]):
        lam += _gauss_bin_mean(theta[k], theta[k + 1], abs(theta[k + 2]), a, b)
        k += 3
    if spec["kind"] == GAUSS_POLY:
        if spec["poly_degree"] >= 0:
            lam += _poly_bin_mean(theta[k:k + spec["poly_degree"] + 1], spec["t_shift"],
                                  spec["t_scale"], a, b)
    else:
        lam += _exp_bin_mean(theta[k], theta[k + 1], spec["t_shift"], spec["t_scale"], a, b)
    return lam


def intensity_2d(theta, nx, ny, xr, yr):
    """2x2 Gauss-Legendre average of A exp(-Q/2) + c over every bin, [ny, nx]."""
    A, mx, my, sx, sy, rho, c = theta
    hx = (xr[1] - xr[0]) / nx
    hy = (yr[1] - yr[0]) / ny
    g = 0.5 / math.sqrt(3.0)
    out = np.zeros((ny, nx), dtype=np.float64)
    xc = xr[0] + (np.arange(nx) + 0.5) * hx
    yc = yr[0] + (np.arange(ny) + 0.5) * hy
    one_m_r2 = 1.0 - rho * rho
    for ox in (-g, g):
        for oy in (-g, g):
            u = (xc + ox * hx - mx) / sx
            v = (yc + oy * hy - my) / sy
            q = (u[None, :] ** 2 - 2.0 * rho * v[:, None] * u[None, :] + v[:, None] ** 2) / one_m_r2
            out += 0.25 * np.exp(-0.5 * q)
    return A * out + c


def poisson_counts(lam, rng) -> np.ndarray:
    return rng.poisson(lam).astype(np.uint32)


def perturb(theta, rel, rng):
    """theta * (1 + rel * N(0,1)) elementwise: an evaluation point off the optimum."""
    theta = np.asarray(theta, dtype=np.float64)
    return theta * (1.0 + rel * rng.standard_normal(theta.shape))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def single_fit_case(seed=1, nbins=10_000):
    """10,000 bins on [0,10]; A Gauss(m=5, s=0.5) + b0 + b1 x with A=1e4, b0=50,
    b1=-2; Poisson counts.  Start point for fits: (8e3, 4.8, 0.6, 45, -1.5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = model_spec(GAUSS_POLY, 1, 1, 0.0, 1.0)
    theta = np.array([1e4, 5.0, 0.5, 50.0, -2.0])
    lam = intensity_1d(spec, theta, nbins, 0.0, 10.0)
    return dict(spec=spec, counts=poisson_counts(lam, rng), range=(0.0, 10.0), theta_true=theta,
                theta0=np.array([8e3, 4.8, 0.6, 45.0, -1.5]))


def large_fit_theta(seed=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.uniform(1e3, 1e5, 2)
    m = rng.uniform(10.0, 90.0, 2)
    s = rng.uniform(0.5, 3.0, 2)
    th = np.array([A[0], m[0], s[0], A[1], m[1], s[1], 100.0, -20.0, 10.0, 5.0])
    return th, rng


def large_fit_case(seed=2, nbins=10_000_000, want_counts=True):
    """1e7 bins on [0,100]: two Gaussians (A ~ U[1e3,1e5], m ~ U[10,90],
    s ~ U[0.5,3]) + cubic c0..c3 = (100,-20,10,5) in t = (x-50)/50.  The
    evaluation point is theta_true * (1 + 0.01 N(0,1)) so the gradient is
    not zero."""
    spec = model_spec(GAUSS_POLY, 2, 3, 50.0, 50.0)
    theta, rng = large_fit_theta(seed)
    out = dict(spec=spec, range=(0.0, 100.0), theta_true=theta, nbins=nbins)
    if want_counts:
        lam = intensity_1d(spec, theta, nbins, 0.0, 100.0)
        out["counts"] = poisson_counts(lam, rng)
    out["theta_eval"] = perturb(theta, 0.01, np.random.Generator(np.random.PCG64(seed + 1000)))
    return out


def batch_case(seed=3, B=4096, lo_bins=256, hi_bins=65536):
    """B independent histograms on [0,1] with nbins log-uniform in
    [lo_bins, hi_bins]; each Gauss (A log-uniform in [1e2,1e4] counts/bin at
    the peak, m ~ U[0,1], s ~ U[0.01,0.05]) + exp(b0 + b1 x) with the
    background at both ends log-uniform in [10,1000] counts/bin."""
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = model_spec(GAUSS_EXP, 1, -1, 0.0, 1.0)
    nb = np.rint(np.exp(rng.uniform(math.log(lo_bins), math.log(hi_bins), B))).astype(np.int64)
    A = np.exp(rng.uniform(math.log(1e2), math.log(1e4), B))
    m = rng.uniform(0.0, 1.0, B)
    s = rng.uniform(0.01, 0.05, B)
    bk0 = np.exp(rng.uniform(math.log(10.0), math.log(1000.0), B))
    bk1 = np.exp(rng.uniform(math.log(10.0), math.log(1000.0), B))
    theta = np.stack([A, m, s, np.log(bk0), np.log(bk1 / bk0)], axis=1)
    offsets = np.zeros(B + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(nb)
    counts = np.empty(offsets[-1], dtype=np.uint32)
    for b in range(B):
        lam = intensity_1d(spec, theta[b], int(nb[b]), 0.0, 1.0)
        counts[offsets[b]:offsets[b + 1]] = poisson_counts(lam, rng)
    ranges = np.tile(np.array([0.0, 1.0]), (B, 1))
    return dict(spec=spec, counts=counts, offsets=offsets, ranges=ranges, theta_true=theta, nbins=nb)


def hist2d_case(seed=4, n=2048):
    """n x n bins on [0,1]^2: A = 1e3, mx,my ~ U[0.3,0.7], sx,sy ~ U[0.05,0.15],
    rho ~ U[-0.5,0.5], c = 10; per-bin float32 weights ~ U[0.5,1.5]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    spec = model_spec(GAUSS2D)
    mx, my = rng.uniform(0.3, 0.7, 2)
    sx, sy = rng.uniform(0.05, 0.15, 2)
    rho = rng.uniform(-0.5, 0.5)
    theta = np.array([1e3, mx, my, sx, sy, rho, 10.0])
    lam = intensity_2d(theta, n, n, (0.0, 1.0), (0.0, 1.0))
    counts = poisson_counts(lam, rng)
    w = rng.uniform(0.5, 1.5, (n, n)).astype(np.float32)
    theta_eval = perturb(theta, 0.01, rng)
    return dict(spec=spec, counts=counts, weights=w, range=(0.0, 1.0, 0.0, 1.0), theta_true=theta,
                theta_eval=theta_eval)


def fig2a_case(seed=5, nbins=1000, entries=100_000):
    """The paper's Fig. 2a workload: 1000 bins on [-5,5] filled with 1e5
    entries drawn from gaus {Constant=100, Mean=1, Sigma=3} as a pdf over the
    histogram range (a multinomial over the bins)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    e = _edges(-5.0, 5.0, nbins)
    p = _gauss_bin_mean(1.0, 1.0, 3.0, e[:-1], e[1:])
    p = p / p.sum()
    counts = rng.multinomial(entries, p).astype(np.uint32)
    spec = model_spec(GAUSS_POLY, 1, -1)
    return dict(spec=spec, counts=counts, range=(-5.0, 5.0), theta0=np.array([100.0, 1.0, 3.0]))


def random_1d_case(spec, nbins, lo, hi, theta, seed, rel=0.02):
    """Poisson counts for an arbitrary 1D model plus a perturbed evaluation point."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = intensity_1d(spec, np.asarray(theta, dtype=np.float64), nbins, lo, hi)
    counts = poisson_counts(lam, rng)
    return dict(spec=spec, counts=counts, range=(lo, hi), theta_true=np.asarray(theta, float),
                theta_eval=perturb(theta, rel, rng))


def kgauss_batch_case(K, seed=6, B=512, nbins=10_000):
    """B histograms of nbins bins on [0,1], each K Gaussians (A log-uniform
    in [3e2, 3e3] counts/bin, means spread over [0.1, 0.9] with a U(-0.02,
    0.02) jitter, s ~ U[0.01, 0.03]) on a linear background b0 + b1 x (b0 ~
    U[20, 200] counts/bin, b1 ~ U[-0.5, 0.5] b0); starts: A and s scaled by
    1 + 0.1 N(0,1), means moved by 0.5 s N(0,1), b0 by 1 + 0.05 N(0,1), b1
    moved by 0.05 b0 N(0,1).  The workload of the gradient comparison (the
    number of parameters grows with K, P = 3K + 2)."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + K))
    spec = model_spec(GAUSS_POLY, K, 1, 0.0, 1.0)
    P = 3 * K + 2
    theta = np.empty((B, P))
    th0 = np.empty((B, P))
    counts = np.empty(B * nbins, dtype=np.uint32)
    centres = np.linspace(0.1, 0.9, K) if K > 1 else np.array([0.5])
    for b in range(B):
        A = np.exp(rng.uniform(math.log(3e2), math.log(3e3), K))
        m = centres + rng.uniform(-0.02, 0.02, K)
        s = rng.uniform(0.01, 0.03, K)
        b0 = rng.uniform(20.0, 200.0)
        b1 = rng.uniform(-0.5, 0.5) * b0
        t = np.empty(P)
        t[0:3 * K:3], t[1:3 * K:3], t[2:3 * K:3] = A, m, s
        t[3 * K], t[3 * K + 1] = b0, b1
        theta[b] = t
        counts[b * nbins:(b + 1) * nbins] = poisson_counts(intensity_1d(spec, t, nbins, 0.0, 1.0), rng)
        z = t.copy()
        z[0:3 * K:3] *= 1 + 0.1 * rng.standard_normal(K)
        z[1:3 * K:3] += 0.5 * s * rng.standard_normal(K)
        z[2:3 * K:3] *= 1 + 0.1 * rng.standard_normal(K)
        z[3 * K] *= 1 + 0.05 * rng.standard_normal()
        z[3 * K + 1] += 0.05 * b0 * rng.standard_normal()
        th0[b] = z
    offsets = np.arange(B + 1, dtype=np.int64) * nbins
    ranges = np.tile(np.array([0.0, 1.0]), (B, 1))
    return dict(spec=spec, counts=counts, offsets=offsets, ranges=ranges, theta_true=theta, theta0=th0)


def batch_case_device(seed, B, nbins=4096, device="cuda"):
    """The batched-fit distribution (see batch_case) with a fixed bin count,
    generated on a torch device: parameters from a seeded CPU generator,
    bin-integrated intensities and Poisson draws on the device (seeded).
    Returns int32 counts (u32 values) of shape [B * nbins], int64 offsets,
    f64 ranges [B, 2] and the generating theta [B, 5] (CPU float64)."""
    import torch

    g = torch.Generator(device="cpu").manual_seed(seed)

    def logu(a, b):
        return torch.exp(torch.empty(B, dtype=torch.float64).uniform_(math.log(a), math.log(b),
                                                                       generator=g))

    A = logu(1e2, 1e4)
    m = torch.empty(B, dtype=torch.float64).uniform_(0.0, 1.0, generator=g)
    s = torch.empty(B, dtype=torch.float64).uniform_(0.01, 0.05, generator=g)
    bk0, bk1 = logu(10.0, 1000.0), logu(10.0, 1000.0)
    theta = torch.stack([A, m, s, torch.log(bk0), torch.log(bk1 / bk0)], dim=1)
    th = theta.to(device)
    e = torch.linspace(0.0, 1.0, nbins + 1, dtype=torch.float64, device=device)
    a, b = e[:-1][None, :], e[1:][None, :]
    h = 1.0 / nbins
    za = (a - th[:, 1:2]) / th[:, 2:3]
    zb = (b - th[:, 1:2]) / th[:, 2:3]
    right = za >= 0
    p = torch.where(right, torch.special.ndtr(-za) - torch.special.ndtr(-zb),
                    torch.special.ndtr(zb) - torch.special.ndtr(za))
    lam = th[:, 0:1] * th[:, 2:3] * math.sqrt(2.0 * math.pi) * p / h
    b1 = th[:, 4:5]
    lam = lam + torch.exp(th[:, 3:4] + b1 * a) * torch.expm1(b1 * h) / (b1 * h)
    gd = torch.Generator(device=device).manual_seed(seed + 7919)
    counts = torch.poisson(lam, generator=gd).to(torch.int32).reshape(-1)
    offsets = torch.arange(B + 1, dtype=torch.int64) * nbins
    ranges = torch.tensor([[0.0, 1.0]], dtype=torch.float64).repeat(B, 1)
    return counts, offsets, ranges, theta


def unbinned_events(spec, theta, lo, hi, n_events, seed, grid=1 << 20):
    """n_events positions drawn from the 1D intensity (as a density on
    [lo, hi]) by inverting its cumulative integral on a fine grid: the bin
    means of the intensity on `grid` bins give the cell probabilities, and a
    uniform draw places each event inside its cell."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lam = np.maximum(intensity_1d(spec, np.asarray(theta, dtype=np.float64), grid, lo, hi), 0.0)
    cdf = np.cumsum(lam)
    cdf /= cdf[-1]
    u = rng.random(n_events)
    cell = np.minimum(np.searchsorted(cdf, u, side="right"), grid - 1)
    h = (hi - lo) / grid
    return lo + (cell + rng.random(n_events)) * h


def unbinned_case(seed=7, n_events=10_000_000):
    """The 1e7-bin workload's model as an intensity on [0, 100]: two
    Gaussians + cubic, n_events positions drawn from it, evaluated at
    theta * (1 + 0.01 N(0,1)) so that the gradient is not zero."""
    spec = model_spec(GAUSS_POLY, 2, 3, 50.0, 50.0)
    theta, rng = large_fit_theta(2)
    x = unbinned_events(spec, theta, 0.0, 100.0, n_events, seed)
    return dict(spec=spec, range=(0.0, 100.0), events=x, theta_true=theta,
                theta_eval=perturb(theta, 0.01, np.random.Generator(np.random.PCG64(seed + 1000))))

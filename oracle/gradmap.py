"""FP64 numpy oracle of the elementwise Gaussian gradient map (test
infrastructure only).

TEST INFRASTRUCTURE ONLY: used by the tests and nothing else; it shares no
code with the HIP kernels.

The function is the device function of paper sec. 3, Listing 1: a Gaussian
of x with mean p and width sigma, normalised by (2 pi)^(-1/2) sigma^(-a).
The listing prints sigma^(-1/2), so a = 1/2 is its reading; a = 1 (the normal
pdf) is offered beside it.  Its gradient with respect to the chosen inputs
is what the listing's generated function returns, one element per thread.

The reverse sweep below follows the forward statements backwards, as a
source transformer would:
    d = x - p;  t = -d^2 / (2 s^2);  e = exp(t);  c = (2 pi)^(-1/2) s^(-a);
    g = c e
with upstream adjoint w:
    e_bar = w c,  c_bar = w e,  t_bar = e_bar e,
    d_bar = t_bar (-d / s^2),  x_bar = d_bar,  p_bar = -d_bar,
    s_bar = t_bar (d^2 / s^3) + c_bar (-a c / s).
A shared input's adjoint is the sum of the per-element adjoints, summed
exactly rounded (math.fsum).
"""
from __future__ import annotations

import math

import numpy as np

NORM_LISTING, NORM_PDF = 0, 1


def norm_exponent(norm: int) -> float:
    return 0.5 if norm == NORM_LISTING else 1.0


def gauss(x, p, sigma, norm=NORM_LISTING):
    """The forward function, elementwise (p and sigma broadcast)."""
    x = np.asarray(x, dtype=np.float64)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), x.shape)
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), x.shape)
    a = norm_exponent(norm)
    d = x - p
    t = -d * d / (2.0 * s * s)
    return (2.0 * math.pi) ** -0.5 * s ** -a * np.exp(t)


def grad_map(x, p, sigma, norm=NORM_LISTING, seed=None):
    """Per-element (g, x_bar, p_bar, s_bar) with upstream adjoints `seed`
    (ones when None)."""
    x = np.asarray(x, dtype=np.float64)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), x.shape)
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64), x.shape)
    w = np.ones_like(x) if seed is None else np.asarray(seed, dtype=np.float64)
    a = norm_exponent(norm)
    # forward sweep
    d = x - p
    t = -d * d / (2.0 * s * s)
    e = np.exp(t)
    c = (2.0 * math.pi) ** -0.5 * s ** -a
    g = c * e
    # reverse sweep
    e_bar = w * c
    c_bar = w * e
    t_bar = e_bar * e
    d_bar = t_bar * (-d / (s * s))
    x_bar = d_bar
    p_bar = -d_bar
    s_bar = t_bar * (d * d / (s * s * s)) + c_bar * (-a * c / s)
    return g, x_bar, p_bar, s_bar


def shared_sum(v) -> float:
    """The adjoint of an input shared by every element."""
    return math.fsum(np.asarray(v, dtype=np.float64).tolist())

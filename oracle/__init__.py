"""FP64 CPU oracle for the binned histogram-fit objective (test infrastructure).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  The
oracle shares no code with the HIP implementation.

Wraps ``liboracle.so`` (built from ``histfit_oracle.c`` by :func:`build`) with
numpy in and out.  Function and argument meanings are documented in the C
source; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "histfit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NEYMAN, PEARSON, POISSON = 0, 1, 2
GAUSS_POLY, GAUSS_EXP, GAUSS2D = 1, 2, 3
ST_DOMAIN, ST_NONFINITE = 1, 2
FIT_CONVERGED, FIT_MAXITER, FIT_LSFAIL, FIT_NONFINITE, FIT_DOMAIN = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (strict IEEE: no fast-math, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=gnu11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class _Model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_gauss", ctypes.c_int32),
                ("poly_degree", ctypes.c_int32), ("bin_average", ctypes.c_int32),
                ("t_shift", ctypes.c_double), ("t_scale", ctypes.c_double)]


class _FitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("ls_max", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("free_mask", ctypes.c_uint32),
                ("edm_tol", ctypes.c_double), ("hessian_init", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


@dataclass(frozen=True)
class Model:
    """Model descriptor: kind 1 = Gaussians + polynomial, 2 = Gaussians +
    exponential background, 3 = 2D correlated Gaussian + constant.
    bin_average (kind 1): mu_i is the model's average over bin i instead of
    its value at the bin centre."""
    kind: int
    n_gauss: int = 1
    poly_degree: int = -1
    t_shift: float = 0.0
    t_scale: float = 1.0
    bin_average: int = 0

    def c(self) -> _Model:
        return _Model(self.kind, self.n_gauss, self.poly_degree, self.bin_average, self.t_shift,
                      self.t_scale)


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        mp = ctypes.POINTER(_Model)
        L.or_nparams.argtypes = [mp]
        L.or_nparams.restype = ctypes.c_int
        L.or_neumaier_sum.argtypes = [dp, ctypes.c_int64]
        L.or_neumaier_sum.restype = ctypes.c_double
        L.or_model_eval.argtypes = [mp, dp, ctypes.c_int64, ctypes.c_int64, dp, dp]
        L.or_model_eval.restype = ctypes.c_int
        L.or_nll_grad_mt.argtypes = [mp, ctypes.c_int, dp, dp, ctypes.c_int64, ctypes.c_int64, dp,
                                     dp, dp, dp, dp, dp, ip, ctypes.c_int]
        L.or_nll_grad_mt.restype = ctypes.c_int
        L.or_fisher.argtypes = [mp, ctypes.c_int, dp, dp, ctypes.c_int64, ctypes.c_int64, dp, dp, dp]
        L.or_fisher.restype = ctypes.c_int
        L.or_fit_mt.argtypes = [mp, ctypes.c_int, dp, dp, ctypes.c_int64, ctypes.c_int64, dp, dp,
                                ctypes.POINTER(_FitOpts), dp, dp, ip, ip, ip, ctypes.c_int]
        L.or_fit_mt.restype = ctypes.c_int
        L.or_fit_many.argtypes = [mp, ctypes.c_int, ctypes.c_int32, dp, lp, dp, dp,
                                  ctypes.POINTER(_FitOpts), dp, dp, ip, ip, ip, ctypes.c_int]
        L.or_fit_many.restype = ctypes.c_int
        L.or_nll_grad_edges.argtypes = [mp, ctypes.c_int, dp, dp, ctypes.c_int64, dp, dp, dp, dp,
                                        dp, dp, ip, ctypes.c_int]
        L.or_nll_grad_edges.restype = ctypes.c_int
        L.or_unbinned.argtypes = [mp, dp, dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  dp, dp, dp, dp, ip]
        L.or_unbinned.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _range4(range4):
    r = np.zeros(4, dtype=np.float64)
    r[: len(range4)] = range4
    if len(range4) == 2:
        r[2:] = (0.0, 1.0)
    return r


def nparams(model: Model) -> int:
    m = model.c()
    return lib().or_nparams(ctypes.byref(m))


def neumaier_sum(v) -> float:
    v = _f64(v)
    return lib().or_neumaier_sum(_dp(v), v.size)


def fisher(model: Model, objective: int, counts, theta, range4, weights=None):
    """Expected Hessian F = sum_i w_i c_i (dmu_i/dtheta)(dmu_i/dtheta)^T
    (c_i = d2l/dmu2 at n_i = mu_i), P x P."""
    c = np.asarray(counts)
    nx = c.shape[-1]
    ny = c.shape[0] if c.ndim == 2 else 1
    c = _f64(c).reshape(-1)
    w = _f64(np.asarray(weights).reshape(-1)) if weights is not None else None
    P = nparams(model)
    F = np.empty(P * P, dtype=np.float64)
    m = model.c()
    rc = lib().or_fisher(ctypes.byref(m), objective, _dp(c), _dp(w), nx, ny, _dp(_range4(range4)),
                         _dp(_f64(theta)), _dp(F))
    if rc != 0:
        raise ValueError("or_fisher failed: %d" % rc)
    return F.reshape(P, P)


def covariance(F, objective: int, free_mask: int = 0):
    """Parameter covariance from an expected Hessian: cov = 2 UP inv(F) over
    the free parameters (bit k of free_mask set, or all when 0), zero rows and
    columns for fixed ones.  UP is the rise of the objective that defines one
    standard error: 1/2 for the Poisson NLL (written without the factor 2),
    1 for a chi-square.  Returns (cov, ok); ok is False (cov NaN in the free
    block) when the free block is not positive definite."""
    F = np.asarray(F, dtype=np.float64)
    P = F.shape[0]
    free = [k for k in range(P) if free_mask == 0 or (free_mask >> k) & 1]
    cov = np.zeros((P, P))
    Ff = F[np.ix_(free, free)]
    scale = 1.0 if objective == 2 else 2.0
    try:
        np.linalg.cholesky(Ff)
        ok = bool(np.all(np.diag(Ff) > 0))
    except np.linalg.LinAlgError:
        ok = False
    cov[np.ix_(free, free)] = scale * np.linalg.inv(Ff) if ok else np.nan
    return cov, ok


def model_eval(model: Model, theta, shape, range4):
    """mu at every bin centre; shape = (nx,) or (ny, nx)."""
    nx = shape[-1]
    ny = shape[0] if len(shape) == 2 else 1
    th = _f64(theta)
    r = _range4(range4)
    mu = np.empty(nx * ny, dtype=np.float64)
    m = model.c()
    rc = lib().or_model_eval(ctypes.byref(m), _dp(th), nx, ny, _dp(r), _dp(mu))
    if rc != 0:
        raise ValueError("or_model_eval failed: %d" % rc)
    return mu.reshape(shape)


@dataclass
class NllGrad:
    nll: float
    grad: np.ndarray
    scales: np.ndarray  # S_0 then S_1..S_P
    status: int
    ell: np.ndarray | None = None


def nll_grad(model: Model, objective: int, counts, theta, range4, weights=None,
             want_ell: bool = False, nthreads: int = 1) -> NllGrad:
    """NLL, gradient and condition scales; counts may be 1D (nx,) or 2D (ny, nx)."""
    c = np.asarray(counts)
    nx = c.shape[-1]
    ny = c.shape[0] if c.ndim == 2 else 1
    c = _f64(c).reshape(-1)
    w = _f64(np.asarray(weights).reshape(-1)) if weights is not None else None
    th = _f64(theta)
    P = nparams(model)
    if th.size != P:
        raise ValueError("theta has %d values, model needs %d" % (th.size, P))
    r = _range4(range4)
    nll = ctypes.c_double()
    grad = np.empty(P, dtype=np.float64)
    sc = np.empty(P + 1, dtype=np.float64)
    ell = np.empty(c.size, dtype=np.float64) if want_ell else None
    st = ctypes.c_int32()
    m = model.c()
    rc = lib().or_nll_grad_mt(ctypes.byref(m), objective, _dp(c), _dp(w), nx, ny, _dp(r), _dp(th),
                              ctypes.byref(nll), _dp(grad), _dp(sc), _dp(ell), ctypes.byref(st),
                              nthreads)
    if rc != 0:
        raise ValueError("or_nll_grad failed: %d" % rc)
    return NllGrad(nll.value, grad, sc, st.value, ell)


def nll_grad_edges(model: Model, objective: int, counts, edges, theta, weights=None,
                   want_ell: bool = False, nthreads: int = 1) -> NllGrad:
    """NLL, gradient and condition scales of a 1D histogram whose bin i spans
    [edges[i], edges[i+1]] (bins of any widths)."""
    c = _f64(np.asarray(counts).reshape(-1))
    e = _f64(np.asarray(edges).reshape(-1))
    if e.size != c.size + 1:
        raise ValueError("edges must have nbins + 1 values")
    w = _f64(np.asarray(weights).reshape(-1)) if weights is not None else None
    th = _f64(theta)
    P = nparams(model)
    nll = ctypes.c_double()
    grad = np.empty(P, dtype=np.float64)
    sc = np.empty(P + 1, dtype=np.float64)
    ell = np.empty(c.size, dtype=np.float64) if want_ell else None
    st = ctypes.c_int32()
    m = model.c()
    rc = lib().or_nll_grad_edges(ctypes.byref(m), objective, _dp(c), _dp(w), c.size, _dp(e),
                                 _dp(th), ctypes.byref(nll), _dp(grad), _dp(sc), _dp(ell),
                                 ctypes.byref(st), nthreads)
    if rc != 0:
        raise ValueError("or_nll_grad_edges failed: %d" % rc)
    return NllGrad(nll.value, grad, sc, st.value, ell)


def unbinned(model: Model, events, lo, hi, theta, weights=None) -> NllGrad:
    """Extended unbinned NLL  L = integral of lambda over [lo, hi] -
    sum_e w_e ln lambda(x_e), its gradient and condition scales (Gauss +
    polynomial models); events outside [lo, hi] are skipped."""
    x = _f64(np.asarray(events).reshape(-1))
    w = _f64(np.asarray(weights).reshape(-1)) if weights is not None else None
    th = _f64(theta)
    P = nparams(model)
    if th.size != P:
        raise ValueError("theta has %d values, model needs %d" % (th.size, P))
    nll = ctypes.c_double()
    grad = np.empty(P, dtype=np.float64)
    sc = np.empty(P + 1, dtype=np.float64)
    st = ctypes.c_int32()
    m = model.c()
    rc = lib().or_unbinned(ctypes.byref(m), _dp(x), _dp(w), x.size, float(lo), float(hi), _dp(th),
                           ctypes.byref(nll), _dp(grad), _dp(sc), ctypes.byref(st))
    if rc != 0:
        raise ValueError("or_unbinned failed: %d" % rc)
    return NllGrad(nll.value, grad, sc, st.value)


@dataclass
class FitResult:
    theta: np.ndarray
    nll: float
    status: int
    iters: int
    nevals: int


def fit(model: Model, objective: int, counts, theta0, range4, weights=None, max_iter=500,
        edm_tol=1e-10, ls_max=30, fixed_iters=False, free_mask=0, nthreads=1,
        hessian_init=0) -> FitResult:
    c = np.asarray(counts)
    nx = c.shape[-1]
    ny = c.shape[0] if c.ndim == 2 else 1
    c = _f64(c).reshape(-1)
    w = _f64(np.asarray(weights).reshape(-1)) if weights is not None else None
    th0 = _f64(theta0)
    P = nparams(model)
    r = _range4(range4)
    opts = _FitOpts(max_iter, ls_max, 1 if fixed_iters else 0, free_mask, edm_tol, hessian_init, 0)
    out = np.empty(P, dtype=np.float64)
    nll = ctypes.c_double()
    st, it, ne = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    m = model.c()
    rc = lib().or_fit_mt(ctypes.byref(m), objective, _dp(c), _dp(w), nx, ny, _dp(r), _dp(th0),
                         ctypes.byref(opts), _dp(out), ctypes.byref(nll), ctypes.byref(st),
                         ctypes.byref(it), ctypes.byref(ne), nthreads)
    if rc != 0:
        raise ValueError("or_fit failed: %d" % rc)
    return FitResult(out, nll.value, st.value, it.value, ne.value)


def fit_many(model: Model, objective: int, counts_concat, offsets, ranges, theta0, max_iter=500,
             edm_tol=1e-10, ls_max=30, nthreads=1, hessian_init=0):
    """Independent fits of B histograms stored end to end; returns arrays."""
    c = _f64(counts_concat)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    rg = _f64(ranges).reshape(-1)
    th0 = _f64(theta0).reshape(-1)
    B = off.size - 1
    P = nparams(model)
    opts = _FitOpts(max_iter, ls_max, 0, 0, edm_tol, hessian_init, 0)
    out = np.empty(B * P, dtype=np.float64)
    nll = np.empty(B, dtype=np.float64)
    st = np.empty(B, dtype=np.int32)
    it = np.empty(B, dtype=np.int32)
    ne = np.empty(B, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int32)
    m = model.c()
    rc = lib().or_fit_many(ctypes.byref(m), objective, B, _dp(c),
                           off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(rg), _dp(th0),
                           ctypes.byref(opts), _dp(out), _dp(nll), st.ctypes.data_as(ip),
                           it.ctypes.data_as(ip), ne.ctypes.data_as(ip), nthreads)
    if rc != 0:
        raise ValueError("or_fit_many failed: %d" % rc)
    return out.reshape(B, P), nll, st, it, ne

"""MI355X histogram-fit library: Python binding of libhistfit.so.

The binding only marshals arguments: torch tensors supply device memory and
the current HIP stream, and every step of the computation runs in the HIP
kernels behind the C ABI declared in include/histfit.h.  There is no CPU
fallback: if the library is missing or no GPU is visible, the calls raise.

Calls (same names as the C ABI):
  nll_eval(hist, model, theta, objective=POISSON, precision=FP64)
  nll_grad(hist, model, theta, objective=POISSON, precision=FP64, seed=None,
           want_grad_w=False, free_mask=0)
  fit_batch(counts_concat, offsets, ranges, model, theta0, objective=POISSON,
            precision=FP64, **fit options)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhistfit.so")

NEYMAN, PEARSON, POISSON = 0, 1, 2
NORM_LISTING, NORM_PDF = 0, 1
GAUSS_POLY, GAUSS_EXP, GAUSS2D = 1, 2, 3
FP64, FP32_BIN = 0, 1
U32, F32, F64 = 0, 1, 2
ST_DOMAIN, ST_NONFINITE = 1, 2
FIT_CONVERGED, FIT_MAXITER, FIT_LSFAIL, FIT_NONFINITE, FIT_DOMAIN, FIT_BADHIST = range(6)
IDENTITY, FISHER = 0, 1  # fit_batch hessian_init
ADJOINT, FINITE_DIFF = 0, 1  # fit_batch gradient


class HfModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_gauss", ctypes.c_int32),
                ("poly_degree", ctypes.c_int32), ("bin_average", ctypes.c_int32),
                ("t_shift", ctypes.c_double), ("t_scale", ctypes.c_double)]


class HfHist(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("counts_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("xlo", ctypes.c_double), ("xhi", ctypes.c_double),
                ("ylo", ctypes.c_double), ("yhi", ctypes.c_double),
                ("x_edges", ctypes.c_void_p)]


class HfFitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("ls_max", ctypes.c_int32),
                ("fixed_iters", ctypes.c_int32), ("free_mask", ctypes.c_uint32),
                ("edm_tol", ctypes.c_double), ("polish_edm", ctypes.c_double),
                ("hessian_init", ctypes.c_int32), ("gradient", ctypes.c_int32)]


@dataclass(frozen=True)
class Model:
    """Model descriptor (see include/histfit.h for the parameter layout).
    bin_average = 1 (1D Gauss + polynomial, nll_eval / nll_grad): mu_i is the
    model's average over bin i instead of its value at the centre."""
    kind: int
    n_gauss: int = 1
    poly_degree: int = -1
    t_shift: float = 0.0
    t_scale: float = 1.0
    bin_average: int = 0

    def c(self) -> HfModel:
        return HfModel(self.kind, self.n_gauss, self.poly_degree, int(self.bin_average),
                       float(self.t_shift), float(self.t_scale))

    @staticmethod
    def from_spec(spec: dict) -> "Model":
        return Model(spec["kind"], spec.get("n_gauss", 1), spec.get("poly_degree", -1),
                     spec.get("t_shift", 0.0), spec.get("t_scale", 1.0),
                     spec.get("bin_average", 0))

    @property
    def nparams(self) -> int:
        rc = load().hf_model_nparams(ctypes.byref(self.c()))
        if rc < 0:
            raise ValueError("unsupported model %r" % (self,))
        return rc


class HistfitError(RuntimeError):
    pass


_lib = None
_ctx = {}      # (device, stream handle) -> hf_ctx
_pool = {}     # device -> contexts created ahead, not yet given to a stream
_tuning = {}   # device -> (wg_per_cu, cache_bins, block_size) set by fit_set_tuning
_wave_bins = {}  # device -> wave_bins set by fit_set_wave_bins
POOL_SIZE = 4  # spare contexts kept for streams first seen during graph capture


def load():
    """Load libhistfit.so (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- binds libamdhip64 before our library
    if not os.path.exists(LIB_PATH):
        raise HistfitError("libhistfit.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64
    L.hf_ctx_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]
    L.hf_ctx_create.restype = ctypes.c_int
    L.hf_ctx_destroy.argtypes = [vp]
    L.hf_ctx_destroy.restype = None
    L.hf_last_error.argtypes = [vp]
    L.hf_last_error.restype = ctypes.c_char_p
    L.hf_model_nparams.argtypes = [ctypes.POINTER(HfModel)]
    L.hf_model_nparams.restype = ctypes.c_int
    L.nll_eval.argtypes = [vp, ctypes.POINTER(HfHist), ctypes.POINTER(HfModel), i32, i32, vp, vp,
                           vp, vp]
    L.nll_eval.restype = ctypes.c_int
    L.nll_grad.argtypes = [vp, ctypes.POINTER(HfHist), ctypes.POINTER(HfModel), i32, i32, vp, vp,
                           vp, vp, vp, u32, vp, vp]
    L.nll_grad.restype = ctypes.c_int
    L.nll_grad_noalloc.argtypes = [ctypes.POINTER(HfHist), ctypes.POINTER(HfModel), i32, i32, vp,
                                   vp, vp, vp, vp, u32, vp, vp]
    L.nll_grad_noalloc.restype = ctypes.c_int
    L.fit_batch.argtypes = [vp, i32, vp, i32, vp, vp, ctypes.POINTER(HfModel), i32, i32, vp,
                            ctypes.POINTER(HfFitOpts), vp, vp, vp, vp, vp, vp]
    L.fit_batch.restype = ctypes.c_int
    f32 = ctypes.c_float
    L.hf_mlp_nparams.argtypes = []
    L.hf_mlp_nparams.restype = i64
    L.hf_mlp_workspace_bytes.argtypes = [i32]
    L.hf_mlp_workspace_bytes.restype = i64
    L.hf_mlp_workspace_layout.argtypes = [i32, vp]
    L.hf_mlp_workspace_layout.restype = ctypes.c_int
    L.hf_rebin_lognorm.argtypes = [vp, i32, vp, i32, vp, f32, f32, vp, vp]
    L.hf_default_starts.argtypes = [vp, i32, vp, i32, vp, vp, ctypes.POINTER(HfModel), vp, vp]
    L.hf_column_stats.argtypes = [vp, i64, i32, vp, vp, vp, vp]
    L.hf_theta_to_target.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.hf_target_to_theta.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.hf_mlp_forward.argtypes = [vp, i32, vp, vp, vp, vp, i64, vp]
    L.hf_mlp_train_step.argtypes = [vp, i32, vp, vp, vp, i32, f32, f32, vp, vp, vp, vp, vp, i64, vp]
    L.hf_fit_set_tuning.argtypes = [vp, i32, i32, i32]
    L.hf_fit_set_wave_bins.argtypes = [vp, i32]
    L.hf_fit_get_wave_bins.argtypes = [vp]
    L.hf_fit_max_wave_bins.argtypes = [vp, ctypes.POINTER(HfModel), i32, i32]
    L.hf_fit_get_tuning.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                    ctypes.POINTER(i32)]
    L.hf_fit_max_cache_bins.argtypes = [vp, ctypes.POINTER(HfModel), i32, i32]
    L.hf_nll_fisher.argtypes = [vp, ctypes.POINTER(HfHist), ctypes.POINTER(HfModel), i32, vp, vp,
                                vp, vp]
    L.hf_fisher_covariance.argtypes = [vp, i32, i32, i32, vp, ctypes.c_uint32, vp, vp, vp]
    L.hf_gauss_grad_map.argtypes = [vp, i64, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp]
    L.nll_unbinned.argtypes = [vp, vp, vp, i64, ctypes.c_double, ctypes.c_double,
                               ctypes.POINTER(HfModel), vp, vp, vp, vp, vp]
    for fn in (L.nll_unbinned, L.hf_gauss_grad_map, L.hf_nll_fisher, L.hf_fisher_covariance, L.hf_rebin_lognorm, L.hf_default_starts, L.hf_column_stats, L.hf_theta_to_target,
               L.hf_target_to_theta, L.hf_mlp_forward, L.hf_mlp_train_step, L.hf_fit_set_tuning,
               L.hf_fit_get_tuning, L.hf_fit_max_cache_bins, L.hf_fit_set_wave_bins,
               L.hf_fit_get_wave_bins, L.hf_fit_max_wave_bins):
        fn.restype = ctypes.c_int
    _lib = L
    return L


def _new_context(dev):
    import torch
    L = load()
    h = ctypes.c_void_p()
    with torch.cuda.device(dev):
        rc = L.hf_ctx_create(ctypes.byref(h), dev)
    if rc != 0:
        raise HistfitError("hf_ctx_create(%d) failed: %d" % (dev, rc))
    if dev in _tuning:
        _check(L.hf_fit_set_tuning(h, *_tuning[dev]), h)
    if dev in _wave_bins:
        _check(L.hf_fit_set_wave_bins(h, _wave_bins[dev]), h)
    return h


def context(device: int | None = None, stream=None):
    """The library context of (device, stream), kept for the process.  A
    context's scratch (block partials, completion ticket, fit queue) may only
    be used by calls that do not overlap, so every stream gets its own:
    calls serialised on one stream share a context, and calls on different
    streams (a graph captured on a side stream and eager work on the default
    stream included) never do.  Creating a context allocates device memory,
    which a stream being captured into a graph must not do, so calls outside
    capture keep POOL_SIZE spare contexts ready, and a stream first seen
    during capture takes one of them.  `stream` defaults to the device's
    current torch stream."""
    import torch
    load()
    if not torch.cuda.is_available():
        raise HistfitError("no GPU visible: the HIP library has no CPU path")
    dev = torch.cuda.current_device() if device is None else int(device)
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    key = (dev, int(stream))
    h = _ctx.get(key)
    pool = _pool.setdefault(dev, [])
    if h is not None and len(pool) >= POOL_SIZE:
        return h
    capturing = torch.cuda.is_current_stream_capturing()
    if h is None:
        if not pool and capturing:
            raise HistfitError("more than %d streams first used during graph capture on device "
                               "%d (or the device's first call is captured); make one call on "
                               "the stream outside capture first: contexts allocate device "
                               "memory" % (POOL_SIZE, dev))
        h = pool.pop(0) if pool else _new_context(dev)
        _ctx[key] = h
    if not capturing:
        while len(pool) < POOL_SIZE:
            pool.append(_new_context(dev))
    return h


def _check(rc, ctx):
    if rc != 0:
        raise HistfitError("histfit error %d: %s" % (rc, load().hf_last_error(ctx).decode()))


def _dtype_code(t):
    import torch
    if t.dtype == torch.int32 or t.dtype == torch.uint32:
        return U32
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError("counts must be int32/uint32 (read as u32), float32 or float64")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(t, dtype, device, name):
    import torch
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(t, dtype=dtype)
    if t.device.type != "cuda":
        t = t.to(device)
    if t.dtype != dtype:
        t = t.to(dtype)
    if not t.is_contiguous():
        t = t.contiguous()
    return t


def _need(t, name, dtype, numel, device):
    """Raises unless t is a contiguous `dtype` tensor on `device` with at
    least `numel` elements: the kernels index it through a plain pointer."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device != device or t.dtype != dtype \
            or not t.is_contiguous() or t.numel() < numel:
        got = (tuple(t.shape), t.dtype, str(t.device)) if isinstance(t, torch.Tensor) else type(t)
        raise ValueError(f"{name}: need a contiguous {dtype} tensor of >= {numel} elements on "
                         f"{device}, got {got}")
    return t


def _check_offsets(offsets, n_counts):
    """Host-side check that every histogram of a batch lies inside counts."""
    import numpy as np
    import torch
    if isinstance(offsets, torch.Tensor) and offsets.device.type != "cpu":
        return  # device offsets: checked by the caller that built them
    o = np.asarray(offsets.numpy() if isinstance(offsets, torch.Tensor) else offsets, dtype=np.int64)
    if o.ndim != 1 or o.size < 2 or o[0] != 0 or np.any(np.diff(o) < 1) or o[-1] > n_counts:
        raise ValueError("offsets must start at 0, increase strictly and end <= counts size")


@dataclass
class Hist:
    """A histogram on the device: counts [nx] or [ny, nx] (x fastest);
    edges: None (uniform bins on xrange) or a device f64[nx + 1] of ascending
    bin edges (1D bins of any widths)."""
    counts: object
    xrange: tuple
    yrange: tuple = (0.0, 1.0)
    weights: object = None
    edges: object = None

    def c(self) -> HfHist:
        c = self.counts
        nx = c.shape[-1]
        ny = c.shape[0] if c.dim() == 2 else 1
        return HfHist(c.data_ptr(), self.weights.data_ptr() if self.weights is not None else None,
                      nx, ny, _dtype_code(c), 0, float(self.xrange[0]), float(self.xrange[1]),
                      float(self.yrange[0]), float(self.yrange[1]),
                      self.edges.data_ptr() if self.edges is not None else None)


def make_hist(counts, xrange, yrange=(0.0, 1.0), weights=None, device=None, edges=None) -> Hist:
    """Device copies (if needed) of counts, weights and bin edges, contiguous.
    With edges (nx + 1 ascending values) xrange is taken from its ends."""
    import numpy as np
    import torch
    device = device or torch.device("cuda", torch.cuda.current_device())
    if isinstance(counts, np.ndarray):
        arr = np.ascontiguousarray(counts)
        c = torch.from_numpy(arr.view(np.int32) if arr.dtype == np.uint32 else arr)
    else:
        c = counts
    if c.dtype == torch.uint32:
        c = c.view(torch.int32)
    if c.dtype not in (torch.int32, torch.float32, torch.float64):
        c = c.to(torch.float64)
    c = c.to(device).contiguous()
    w = None if weights is None else _dev_tensor(weights, torch.float32, device, "weights")
    e = None
    if edges is not None:
        e = _dev_tensor(edges, torch.float64, device, "edges").reshape(-1)
        if c.dim() != 1 or e.numel() != c.numel() + 1:
            raise ValueError("edges must have nx + 1 values for a 1D histogram")
        ends = e[[0, -1]].cpu().tolist()
        xrange = (ends[0], ends[1])
    return Hist(c, tuple(xrange), tuple(yrange), w, e)


def _check_theta(th, model):
    P = model.nparams
    if th.numel() != P:
        raise ValueError("theta has %d values, the model has %d parameters" % (th.numel(), P))


def _check_hist_sizes(hist: Hist):
    """Raises unless the histogram's tensors are what the kernels read through
    plain pointers: contiguous, on one GPU, of the expected dtypes and sizes
    (counts [nx] or [ny, nx] int32/uint32/f32/f64, weights f32 per bin,
    edges f64[nx + 1] for 1D)."""
    import torch
    c = hist.counts
    if not isinstance(c, torch.Tensor) or c.device.type != "cuda":
        raise ValueError("counts must be a device tensor")
    if c.dim() not in (1, 2):
        raise ValueError("counts must be [nx] or [ny, nx]")
    if c.dtype not in (torch.int32, torch.uint32, torch.float32, torch.float64):
        raise ValueError("counts must be int32/uint32 (read as u32), float32 or float64")
    if not c.is_contiguous():
        raise ValueError("counts must be contiguous")
    if hist.weights is not None:
        w = hist.weights
        if not isinstance(w, torch.Tensor) or w.numel() != c.numel():
            raise ValueError("weights must have one value per bin")
        _need(w, "weights", torch.float32, c.numel(), c.device)
    if hist.edges is not None:
        if c.dim() != 1:
            raise ValueError("edges are for 1D histograms")
        _need(hist.edges, "edges", torch.float64, c.numel() + 1, c.device)
        if hist.edges.numel() != c.numel() + 1:
            raise ValueError("edges must have nx + 1 values")


def nll_eval(hist: Hist, model: Model, theta, objective=POISSON, precision=FP64, out=None,
             status=None):
    """L(theta) as a device f64[1] tensor (and the status word if asked for)."""
    import torch
    _check_hist_sizes(hist)
    dev = hist.counts.device
    ctx = context(dev.index)
    th = _dev_tensor(theta, torch.float64, dev, "theta")
    _check_theta(th, model)
    out = torch.empty(1, dtype=torch.float64, device=dev) if out is None else out
    _need(out, "out", torch.float64, 1, dev)
    if status is not None:
        _need(status, "status", torch.int32, 1, dev)
    rc = load().nll_eval(ctx, ctypes.byref(hist.c()), ctypes.byref(model.c()), objective,
                         precision, _ptr(th), _ptr(out), _ptr(status), _stream(dev))
    _check(rc, ctx)
    return out


def nll_grad(hist: Hist, model: Model, theta, objective=POISSON, precision=FP64, seed=None,
             want_grad_w=False, free_mask=0, nll_out=None, grad_out=None, grad_w_out=None,
             status=None):
    """(L, dL/dtheta * seed, optional seed * dL/dw) as device tensors."""
    import torch
    _check_hist_sizes(hist)
    dev = hist.counts.device
    ctx = context(dev.index)
    th = _dev_tensor(theta, torch.float64, dev, "theta")
    _check_theta(th, model)
    P = th.numel()
    if grad_w_out is not None and grad_w_out.numel() != hist.counts.numel():
        raise ValueError("grad_w_out must have one value per bin")
    nll_out = torch.empty(1, dtype=torch.float64, device=dev) if nll_out is None else nll_out
    grad_out = torch.empty(P, dtype=torch.float64, device=dev) if grad_out is None else grad_out
    if want_grad_w and grad_w_out is None:
        grad_w_out = torch.empty(hist.counts.shape, dtype=torch.float32, device=dev)
    _need(nll_out, "nll_out", torch.float64, 1, dev)
    _need(grad_out, "grad_out", torch.float64, P, dev)
    if grad_w_out is not None:
        _need(grad_w_out, "grad_w_out", torch.float32, hist.counts.numel(), dev)
    if status is not None:
        _need(status, "status", torch.int32, 1, dev)
    sd = None if seed is None else _dev_tensor(seed, torch.float64, dev, "seed")
    if sd is not None and sd.numel() != 1:
        raise ValueError("seed must hold one value")
    rc = load().nll_grad(ctx, ctypes.byref(hist.c()), ctypes.byref(model.c()), objective,
                         precision, _ptr(th), _ptr(sd), _ptr(nll_out), _ptr(grad_out),
                         _ptr(grad_w_out), free_mask, _ptr(status), _stream(dev))
    _check(rc, ctx)
    return nll_out, grad_out, grad_w_out


def nll_fisher(hist: Hist, model: Model, theta, objective=POISSON, out=None, status=None):
    """Expected Hessian F = sum_i w_i c_i (dmu_i/dtheta)(dmu_i/dtheta)^T at
    theta as a device f64[P, P] tensor (c_i = 1/mu Poisson, 2/mu Pearson,
    2/n Neyman)."""
    import torch
    _check_hist_sizes(hist)
    dev = hist.counts.device
    ctx = context(dev.index)
    th = _dev_tensor(theta, torch.float64, dev, "theta")
    _check_theta(th, model)
    P = th.numel()
    if out is None:
        out = torch.empty((P, P), dtype=torch.float64, device=dev)
    elif out.numel() != P * P:
        raise ValueError("out must be a contiguous f64 tensor of P*P values")
    _need(out, "out", torch.float64, P * P, dev)
    if status is not None:
        _need(status, "status", torch.int32, 1, dev)
    rc = load().hf_nll_fisher(ctx, ctypes.byref(hist.c()), ctypes.byref(model.c()), objective,
                              _ptr(th), _ptr(out), _ptr(status), _stream(dev))
    _check(rc, ctx)
    return out


def fisher_covariance(fisher, objective=POISSON, free_mask=0, out=None, status=None):
    """Covariance 2 UP F^-1 over the free parameters of each [P, P] Fisher
    matrix in `fisher` ([P, P] or [B, P, P], device f64); UP = 1/2 for the
    Poisson NLL, 1 for the chi-squares.  Returns (cov, status) with status
    1 where the free block is not positive definite (cov NaN there)."""
    import torch
    F = fisher
    if F.dtype != torch.float64 or F.dim() not in (2, 3) or F.shape[-1] != F.shape[-2]:
        raise ValueError("fisher must be f64 [P, P] or [B, P, P]")
    F = F.contiguous()
    dev = F.device
    ctx = context(dev.index)
    P = F.shape[-1]
    B = 1 if F.dim() == 2 else F.shape[0]
    out = torch.empty_like(F) if out is None else out
    if out.shape != F.shape or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous f64 tensor shaped like fisher")
    status = torch.empty(B, dtype=torch.int32, device=dev) if status is None else status
    rc = load().hf_fisher_covariance(ctx, B, P, objective, _ptr(F), free_mask, _ptr(out),
                                     _ptr(status), _stream(dev))
    _check(rc, ctx)
    return out, status


def nll_unbinned(events, lo, hi, model: Model, theta, weights=None, want_grad=True, nll_out=None,
                 grad_out=None, status=None):
    """Extended unbinned NLL  Lambda - sum_e w_e ln lambda(x_e)  of the events
    (device f64[n]) in [lo, hi] and, if want_grad, its gradient; device
    tensors (nll, grad or None)."""
    import torch
    if not isinstance(events, torch.Tensor) or events.dtype != torch.float64 or events.dim() != 1:
        raise ValueError("events must be a 1-D f64 tensor")
    dev = events.device
    ctx = context(dev.index)
    ev = events.contiguous()
    th = _dev_tensor(theta, torch.float64, dev, "theta")
    _check_theta(th, model)
    w = None if weights is None else _dev_tensor(weights, torch.float32, dev, "weights")
    if w is not None and w.numel() != ev.numel():
        raise ValueError("weights must have one value per event")
    nll_out = torch.empty(1, dtype=torch.float64, device=dev) if nll_out is None else nll_out
    if want_grad and grad_out is None:
        grad_out = torch.empty(th.numel(), dtype=torch.float64, device=dev)
    rc = load().nll_unbinned(ctx, _ptr(ev), _ptr(w), ev.numel(), float(lo), float(hi),
                             ctypes.byref(model.c()), _ptr(th), _ptr(nll_out),
                             _ptr(grad_out if want_grad else None), _ptr(status), _stream(dev))
    _check(rc, ctx)
    return nll_out, (grad_out if want_grad else None)


def gauss_grad_map(x, p, sigma, norm=NORM_LISTING, seed=None, want_g=True, want_dx=True,
                   want_dp=True, want_dsigma=False):
    """Elementwise g_i = (2 pi)^(-1/2) s^(-a) exp(-(x_i - p_i)^2 / (2 s^2)) and
    its reverse-mode gradient with upstream adjoints `seed` (device f64[n] or
    None for 1).  x is a device f64[n]; p and sigma are device f64[n] or a
    single value (shared by every element, whose adjoint is then the sum over
    the elements).  Returns (g, dx, dp, dsigma), None for the ones not asked
    for."""
    import torch
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or x.dim() != 1:
        raise ValueError("x must be a 1-D f64 tensor")
    dev = x.device
    ctx = context(dev.index)
    n = x.numel()
    x = x.contiguous()
    p = _dev_tensor(p, torch.float64, dev, "p").reshape(-1).contiguous()
    s = _dev_tensor(sigma, torch.float64, dev, "sigma").reshape(-1).contiguous()
    psh, ssh = int(p.numel() == 1), int(s.numel() == 1)
    for name, t in (("p", p), ("sigma", s)):
        if t.numel() not in (1, n):
            raise ValueError("%s must have 1 or n values" % name)
    sd = None if seed is None else _dev_tensor(seed, torch.float64, dev, "seed").reshape(-1)
    if sd is not None and sd.numel() != n:
        raise ValueError("seed must have n values")

    def new(k, flag):
        return torch.empty(k, dtype=torch.float64, device=dev) if flag else None

    g, dx = new(n, want_g), new(n, want_dx)
    dp, ds = new(1 if psh else n, want_dp), new(1 if ssh else n, want_dsigma)
    rc = load().hf_gauss_grad_map(ctx, n, _ptr(x), _ptr(p), psh, _ptr(s), ssh, norm, _ptr(sd),
                                  _ptr(g), _ptr(dx), _ptr(dp), _ptr(ds), _stream(dev))
    _check(rc, ctx)
    return g, dx, dp, ds


@dataclass
class FitBatchResult:
    theta: object
    nll: object
    status: object
    iters: object
    nevals: object


def fit_batch(counts_concat, offsets, ranges, model: Model, theta0, objective=POISSON,
              precision=FP64, max_iter=500, ls_max=30, fixed_iters=False, free_mask=0,
              edm_tol=1e-10, polish_edm=0.0, hessian_init=FISHER, gradient=ADJOINT,
              out: FitBatchResult | None = None):
    """Fit B histograms laid end to end in counts_concat; device tensors out.
    hessian_init: IDENTITY or FISHER (inverse expected Hessian at theta0);
    gradient: ADJOINT (reverse-mode sweep) or FINITE_DIFF (central
    differences of the objective, FP64 only)."""
    import torch
    c = counts_concat
    if not isinstance(c, torch.Tensor) or c.device.type != "cuda" or not c.is_contiguous():
        raise ValueError("counts_concat must be a contiguous device tensor")
    dev = c.device
    ctx = context(dev.index)
    if not isinstance(offsets, torch.Tensor) or offsets.device.type == "cpu":
        # host-side check that every histogram lies inside counts_concat
        import numpy as np
        o = np.asarray(offsets.numpy() if isinstance(offsets, torch.Tensor) else offsets,
                       dtype=np.int64)
        if o.ndim != 1 or o.size < 1 or o[0] != 0 or np.any(np.diff(o) < 0) or o[-1] > c.numel():
            raise ValueError("offsets must start at 0, be nondecreasing and end <= counts size")
    off = _dev_tensor(offsets, torch.int64, dev, "offsets")
    rg = _dev_tensor(ranges, torch.float64, dev, "ranges")
    B = off.numel() - 1
    P = model.nparams
    th0 = _dev_tensor(theta0, torch.float64, dev, "theta0")
    if th0.numel() != B * P or rg.numel() != 2 * B:
        raise ValueError("theta0 must be [B, P] and ranges [B, 2]")
    if out is None:
        out = FitBatchResult(torch.empty(B, P, dtype=torch.float64, device=dev),
                             torch.empty(B, dtype=torch.float64, device=dev),
                             torch.empty(B, dtype=torch.int32, device=dev),
                             torch.empty(B, dtype=torch.int32, device=dev),
                             torch.empty(B, dtype=torch.int32, device=dev))
    _need(out.theta, "out.theta", torch.float64, B * P, dev)
    _need(out.nll, "out.nll", torch.float64, B, dev)
    for name in ("status", "iters", "nevals"):
        _need(getattr(out, name), "out." + name, torch.int32, B, dev)
    opts = HfFitOpts(max_iter, ls_max, 1 if fixed_iters else 0, free_mask, edm_tol, polish_edm,
                     int(hessian_init), int(gradient))
    rc = load().fit_batch(ctx, B, _ptr(c), _dtype_code(c), _ptr(off), _ptr(rg),
                          ctypes.byref(model.c()), objective, precision, _ptr(th0),
                          ctypes.byref(opts), _ptr(out.theta), _ptr(out.nll), _ptr(out.status),
                          _ptr(out.iters), _ptr(out.nevals), _stream(dev))
    _check(rc, ctx)
    return out


def fit_set_tuning(wg_per_cu: int, cache_bins: int, block_size: int = 256, device=None):
    """fit_batch launch shape (see hf_fit_set_tuning) of every context of the
    device, those of streams first used later included."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    shape = (int(wg_per_cu), int(cache_bins), int(block_size))
    ctx = context(dev)
    _check(load().hf_fit_set_tuning(ctx, *shape), ctx)
    _tuning[dev] = shape
    others = [h for (d, _), h in _ctx.items() if d == dev] + _pool.get(dev, [])
    for h in others:
        if h is not ctx:
            _check(load().hf_fit_set_tuning(h, *shape), h)


def fit_set_wave_bins(wave_bins: int, device=None):
    """One wave per histogram of at most wave_bins bins in fit_batch (see
    hf_fit_set_wave_bins; 0 turns it off) on every context of the device."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    ctx = context(dev)
    _check(load().hf_fit_set_wave_bins(ctx, int(wave_bins)), ctx)
    _wave_bins[dev] = int(wave_bins)
    others = [h for (d, _), h in _ctx.items() if d == dev] + _pool.get(dev, [])
    for h in others:
        if h is not ctx:
            _check(load().hf_fit_set_wave_bins(h, int(wave_bins)), h)


def fit_get_wave_bins(device=None) -> int:
    return int(load().hf_fit_get_wave_bins(context(device)))


def fit_max_wave_bins(model: Model, objective=POISSON, block_size: int = 256, device=None) -> int:
    ctx = context(device)
    rc = load().hf_fit_max_wave_bins(ctx, ctypes.byref(model.c()), objective, int(block_size))
    _check(rc if rc < 0 else 0, ctx)
    return rc


def fit_get_tuning(device=None):
    """(wg_per_cu, cache_bins, block_size) of the device's current-stream context."""
    ctx = context(device)
    w, c, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().hf_fit_get_tuning(ctx, ctypes.byref(w), ctypes.byref(c), ctypes.byref(b)), ctx)
    return w.value, c.value, b.value


def fit_max_cache_bins(model: Model, objective=POISSON, block_size: int = 256, device=None) -> int:
    ctx = context(device)
    rc = load().hf_fit_max_cache_bins(ctx, ctypes.byref(model.c()), objective, int(block_size))
    _check(rc if rc < 0 else 0, ctx)
    return rc


# ---------------------------------------------------------------------------
# Learned initialiser (see include/histfit.h for the definitions)
# ---------------------------------------------------------------------------
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_OUT_PAD = 256, 512, 5, 32


def mlp_nparams() -> int:
    return int(load().hf_mlp_nparams())


def mlp_workspace(batch: int, device):
    import torch
    n = int(load().hf_mlp_workspace_bytes(batch))
    if n < 0:
        raise ValueError("batch must be a positive multiple of 64")
    return torch.empty(n, dtype=torch.uint8, device=device)


def mlp_workspace_views(workspace, batch: int) -> dict:
    """Views of the values a workspace stores (see hf_mlp_workspace_layout):
    'a0'..'a3' and 'dz1'..'dz4' as int16 tensors holding BF16 bit patterns,
    'z1'..'z3' and 'y' as float32, each [batch][columns]."""
    import torch
    offs = (ctypes.c_int64 * 12)()
    rc = load().hf_mlp_workspace_layout(int(batch), offs)
    if rc != 0:
        raise ValueError("batch must be a positive multiple of 64")
    ins = (MLP_IN, MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN)
    outs = (MLP_HIDDEN, MLP_HIDDEN, MLP_HIDDEN, MLP_OUT_PAD)
    spec = [("a%d" % l, torch.int16, ins[l]) for l in range(4)]
    spec += [("z%d" % l, torch.float32, MLP_HIDDEN) for l in (1, 2, 3)]
    spec += [("y", torch.float32, MLP_OUT_PAD)]
    spec += [("dz%d" % l, torch.int16, outs[l - 1]) for l in (1, 2, 3, 4)]
    views = {}
    for (name, dt, cols), o in zip(spec, offs):
        nbytes = batch * cols * (2 if dt == torch.int16 else 4)
        if o + nbytes > workspace.numel():
            raise ValueError("workspace too small for batch %d" % batch)
        views[name] = workspace[o:o + nbytes].view(dt).view(batch, cols)
    return views


def _batch_args(counts_concat, offsets):
    import torch
    c = counts_concat
    if not isinstance(c, torch.Tensor) or c.device.type != "cuda" or not c.is_contiguous():
        raise ValueError("counts_concat must be a contiguous device tensor")
    _check_offsets(offsets, c.numel())
    off = offsets if isinstance(offsets, torch.Tensor) and offsets.device == c.device else \
        _dev_tensor(offsets, torch.int64, c.device, "offsets")
    _need(off, "offsets", torch.int64, 2, c.device)
    return c, off, off.numel() - 1


def rebin_lognorm(counts_concat, offsets, in_mean=0.0, in_std=1.0, out=None):
    import torch
    c, off, B = _batch_args(counts_concat, offsets)
    ctx = context(c.device.index)
    out = torch.empty(B, MLP_IN, dtype=torch.float32, device=c.device) if out is None else out
    _need(out, "out", torch.float32, B * MLP_IN, c.device)
    _check(load().hf_rebin_lognorm(ctx, B, _ptr(c), _dtype_code(c), _ptr(off), float(in_mean),
                                   float(in_std), _ptr(out), _stream(c.device)), ctx)
    return out


def default_starts(counts_concat, offsets, ranges, model: Model, out=None):
    import torch
    c, off, B = _batch_args(counts_concat, offsets)
    ctx = context(c.device.index)
    rg = _need(_dev_tensor(ranges, torch.float64, c.device, "ranges"), "ranges", torch.float64,
               2 * B, c.device)
    out = torch.empty(B, 5, dtype=torch.float64, device=c.device) if out is None else out
    _need(out, "out", torch.float64, B * 5, c.device)
    _check(load().hf_default_starts(ctx, B, _ptr(c), _dtype_code(c), _ptr(off), _ptr(rg),
                                    ctypes.byref(model.c()), _ptr(out), _stream(c.device)), ctx)
    return out


def column_stats(x):
    """Per-column mean and standard deviation of a device f32 [n, cols] tensor."""
    import torch
    x = _dev_tensor(x, torch.float32, x.device, "x")
    n, cols = x.shape
    ctx = context(x.device.index)
    mean = torch.empty(cols, dtype=torch.float32, device=x.device)
    std = torch.empty(cols, dtype=torch.float32, device=x.device)
    _check(load().hf_column_stats(ctx, n, cols, _ptr(x), _ptr(mean), _ptr(std), _stream(x.device)),
           ctx)
    return mean, std


def theta_to_target(theta, mean, std, out=None):
    import torch
    B = theta.shape[0]
    dev = theta.device
    ctx = context(dev.index)
    theta = _need(theta.contiguous(), "theta", torch.float64, B * 5, dev)
    _need(mean, "mean", torch.float32, 5, dev)
    _need(std, "std", torch.float32, 5, dev)
    out = torch.empty(B, 5, dtype=torch.float32, device=dev) if out is None else out
    _need(out, "out", torch.float32, B * 5, dev)
    _check(load().hf_theta_to_target(ctx, B, _ptr(theta), _ptr(mean), _ptr(std),
                                     _ptr(out), _stream(dev)), ctx)
    return out


def target_to_theta(y, mean, std, out=None):
    import torch
    B = y.shape[0]
    ctx = context(y.device.index)
    _need(y, "y", torch.float32, B * MLP_OUT_PAD, y.device)
    _need(mean, "mean", torch.float32, 5, y.device)
    _need(std, "std", torch.float32, 5, y.device)
    out = torch.empty(B, 5, dtype=torch.float64, device=y.device) if out is None else out
    _need(out, "out", torch.float64, B * 5, y.device)
    _check(load().hf_target_to_theta(ctx, B, _ptr(y), _ptr(mean), _ptr(std), _ptr(out),
                                     _stream(y.device)), ctx)
    return out


def mlp_forward(params, x, y=None, workspace=None):
    import torch
    B = x.shape[0]
    ctx = context(x.device.index)
    dev = x.device
    y = torch.empty(B, MLP_OUT_PAD, dtype=torch.float32, device=dev) if y is None else y
    ws = mlp_workspace(B, dev) if workspace is None else workspace
    _need(params, "params", torch.float32, mlp_nparams(), dev)
    _need(x, "x", torch.float32, B * MLP_IN, dev)
    _need(y, "y", torch.float32, B * MLP_OUT_PAD, dev)
    _need(ws, "workspace", torch.uint8, 1, dev)
    _check(load().hf_mlp_forward(ctx, B, _ptr(params), _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                 _stream(dev)), ctx)
    return y


def mlp_train_step(params, adam_m, adam_v, step, lr, wd, x, target, grads, loss, workspace):
    import torch
    B = x.shape[0]
    dev = x.device
    ctx = context(dev.index)
    n = mlp_nparams()
    for t, name in ((params, "params"), (adam_m, "adam_m"), (adam_v, "adam_v"), (grads, "grads")):
        _need(t, name, torch.float32, n, dev)
    _need(x, "x", torch.float32, B * MLP_IN, dev)
    _need(target, "target", torch.float32, B * MLP_OUT, dev)
    _need(loss, "loss", torch.float32, 1, dev)
    _need(workspace, "workspace", torch.uint8, 1, dev)
    _check(load().hf_mlp_train_step(ctx, B, _ptr(params), _ptr(adam_m), _ptr(adam_v), int(step),
                                    float(lr), float(wd), _ptr(x), _ptr(target), _ptr(grads),
                                    _ptr(loss), _ptr(workspace), workspace.numel(), _stream(dev)),
           ctx)

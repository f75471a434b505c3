"""GPU parity of hf_gauss_grad_map against the FP64 oracle (oracle/gradmap.py).

Elementwise, with t = -d^2/(2 s^2) the exponent: both sides round t within a
few ulps of |t|, and exp turns an absolute error in t into a relative one, so
  |g - g_ref|   <= 4e-15 (1 + |t|) |g_ref|
  |dx - dx_ref| <= 8e-15 (1 + |t|) |dx_ref|  (and dp = -dx exactly)
  |ds - ds_ref| <= 8e-15 (1 + |t|) |w g| (d^2/s^3 + a/s)   (ds cancels where
                                                            d^2/s^2 = a)
plus an absolute 1e-290 for results below the normal range.
Shared-input adjoints are sums over the elements:
  |S - S_ref| <= 1e-12 sum_i |term_i|.
Sizes cover n = 0, odd tails of the 16-byte pair path, a misaligned (scalar)
path, and 2^27 elements, the bench's size, every element compared.
"""
import numpy as np
import pytest

from oracle import gradmap as og

pytestmark = pytest.mark.gpu

# Far in the tails g is subnormal (t < -708), where one rounding is a large
# relative error: values below the normal range are compared absolutely.
TINY = 1e-290


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-3, 3, n)
    s = rng.uniform(0.3, 2.5, n)
    x = p + s * rng.uniform(-40, 40, n)  # tails down to t = -800 (g underflows to 0)
    x[: n // 3] = p[: n // 3] + s[: n // 3] * rng.uniform(-4, 4, n // 3)
    return x, p, s


def _check_elementwise(got, ref, x, p, s, w, norm):
    g, dx, dp, ds = got
    gr, xr, pr, sr = ref
    d = x - p
    t = np.abs(d * d / (2 * s * s))
    a = og.norm_exponent(norm)
    if g is not None:
        assert np.all(np.abs(g - gr) <= 4e-15 * (1 + t) * np.abs(gr) + TINY), "g"
    if dx is not None:
        assert np.all(np.abs(dx - xr) <= 8e-15 * (1 + t) * np.abs(xr) + TINY), "dx"
    if dp is not None and dx is not None:
        assert np.array_equal(dp, -dx)
    if ds is not None:
        scale = np.abs(w * gr) * (d * d / s ** 3 + a / s)
        assert np.all(np.abs(ds - sr) <= 8e-15 * (1 + t) * scale + TINY), "ds"


def _run(hf, x, p, s, norm, seed, **kw):
    import torch
    dev = "cuda"
    xt = torch.tensor(x, device=dev)
    pt = torch.tensor(np.atleast_1d(p), device=dev)
    st = torch.tensor(np.atleast_1d(s), device=dev)
    wt = None if seed is None else torch.tensor(seed, device=dev)
    out = hf.gauss_grad_map(xt, pt, st, norm=norm, seed=wt, **kw)
    torch.cuda.synchronize()
    return [None if o is None else o.cpu().numpy() for o in out]


@pytest.mark.parametrize("norm", [0, 1])
@pytest.mark.parametrize("n", [1, 2, 3, 511, 512, 513, 100_001])
def test_per_element_parity(hf, n, norm):
    x, p, s = _inputs(n, seed=n)
    w = np.random.default_rng(n + 1).uniform(-2, 2, n)
    for seed in (None, w):
        got = _run(hf, x, p, s, norm, seed, want_dsigma=True)
        ww = np.ones(n) if seed is None else seed
        _check_elementwise(got, og.grad_map(x, p, s, norm, seed), x, p, s, ww, norm)


@pytest.mark.parametrize("shared", ["p", "sigma", "both"])
@pytest.mark.parametrize("n", [1, 7, 4096, 1_000_003])
def test_shared_inputs_reduce(hf, n, shared):
    """The listing's shared sigma, and a shared mean: the shared input's
    adjoint is the sum over the elements; the rest stay per element."""
    x, p, s = _inputs(n, seed=7 * n)
    if shared in ("p", "both"):
        p = np.float64(0.4)
    if shared in ("sigma", "both"):
        s = np.float64(1.3)
    w = np.random.default_rng(n).uniform(-2, 2, n)
    g, dx, dp, ds = _run(hf, x, p, s, 1, w, want_dsigma=True)
    gr, xr, pr, sr = og.grad_map(x, p, s, 1, w)
    pb = np.broadcast_to(p, x.shape)
    sb = np.broadcast_to(s, x.shape)
    _check_elementwise((g, dx, None, None), (gr, xr, pr, sr), x, pb, sb, w, 1)
    if shared in ("p", "both"):
        assert dp.shape == (1,)
        assert abs(dp[0] - og.shared_sum(pr)) <= 1e-12 * np.sum(np.abs(pr)) + 1e-300
    else:
        np.testing.assert_array_equal(dp, -dx)
    if shared in ("sigma", "both"):
        assert ds.shape == (1,)
        assert abs(ds[0] - og.shared_sum(sr)) <= 1e-12 * np.sum(np.abs(sr)) + 1e-300
    else:
        _check_elementwise((None, None, None, ds), (gr, xr, pr, sr), x, pb, sb, w, 1)


def test_misaligned_arrays_and_optional_outputs(hf):
    """Views starting one element in take the scalar path; outputs not asked
    for are not computed."""
    import torch
    n = 1001
    x, p, s = _inputs(n + 1, seed=11)
    xt = torch.tensor(x, device="cuda")[1:]
    pt = torch.tensor(p, device="cuda")[1:]
    st = torch.tensor(s, device="cuda")[1:]
    assert xt.data_ptr() % 16 == 8
    g, dx, dp, ds = hf.gauss_grad_map(xt, pt, st, norm=0, want_g=False, want_dp=False)
    torch.cuda.synchronize()
    assert g is None and dp is None and ds is None
    ref = og.grad_map(x[1:], p[1:], s[1:], 0)
    _check_elementwise((None, dx.cpu().numpy(), None, None), ref, x[1:], p[1:], s[1:],
                       np.ones(n), 0)


def test_empty_and_validation(hf):
    import torch
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    g, dx, dp, ds = hf.gauss_grad_map(e, e, e)
    assert g.numel() == 0 and dx.numel() == 0
    one = torch.tensor([1.0], dtype=torch.float64, device="cuda")
    _, _, dp, ds = hf.gauss_grad_map(e, torch.tensor([0.5], dtype=torch.float64, device="cuda"),
                                     one, want_dsigma=True)
    torch.cuda.synchronize()
    assert dp.item() == 0.0 and ds.item() == 0.0
    with pytest.raises(ValueError):
        hf.gauss_grad_map(torch.zeros(4, dtype=torch.float64, device="cuda"),
                          torch.zeros(3, dtype=torch.float64, device="cuda"), one)
    with pytest.raises(hf.HistfitError):
        hf.gauss_grad_map(torch.zeros(4, dtype=torch.float64, device="cuda"), one, one, norm=5)


@pytest.mark.slow
def test_full_size_in_chunks(hf):
    """2^27 elements (the bench's size, per-element x and p, shared sigma),
    every element compared, in chunks of 2^23; the shared sigma's adjoint
    (a sum over all 2^27 elements) against the FP64 sum of the oracle's
    per-element terms (pairwise summation: error ~27 ulps of sum |terms|,
    far inside the 1e-12 bound)."""
    import torch
    n = 1 << 27
    gen = torch.Generator(device="cuda").manual_seed(12)
    p = torch.rand(n, dtype=torch.float64, device="cuda", generator=gen) * 6 - 3
    x = p + torch.randn(n, dtype=torch.float64, device="cuda", generator=gen) * 2
    s = torch.tensor([1.25], dtype=torch.float64, device="cuda")
    g, dx, dp, ds = hf.gauss_grad_map(x, p, s, norm=0, want_dsigma=True)
    torch.cuda.synchronize()
    chunk = 1 << 23
    tot, tot_abs = 0.0, 0.0
    for c0 in range(0, n, chunk):
        sl = slice(c0, c0 + chunk)
        xs, ps = x[sl].cpu().numpy(), p[sl].cpu().numpy()
        ref = og.grad_map(xs, ps, 1.25, 0)
        got = (g[sl].cpu().numpy(), dx[sl].cpu().numpy(), dp[sl].cpu().numpy(), None)
        _check_elementwise(got, ref, xs, ps, np.full(xs.shape, 1.25), np.ones(xs.size), 0)
        tot += float(np.sum(ref[3]))
        tot_abs += float(np.sum(np.abs(ref[3])))
    assert abs(ds.item() - tot) <= 1e-12 * tot_abs, (ds.item(), tot, tot_abs)
    del x, p, g, dx, dp, ds

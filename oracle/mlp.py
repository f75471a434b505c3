"""FP64 numpy oracle of the learned initialiser (test infrastructure only).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.  It
shares no code with the HIP kernels.

Covers, each as its definition written out:
  * bf16(x): FP64 -> FP32 -> BF16 round to nearest even, back to FP64 (the
    kernels round FP32 values, so the oracle rounds through FP32 first);
  * the dense GELU network 256 -> 512 -> 512 -> 512 -> 5 (output padded to
    32) with the rounding points of the kernels: input, weights, hidden
    activations and the layer adjoints are rounded to BF16 before each
    product; products are summed in FP64 here;
  * its backward pass for loss = sum (y - t)^2 / (5 B), and AdamW
    (Loshchilov & Hutter) with beta1 0.9, beta2 0.999, eps 1e-8;
  * the 256-bin rebinning with log1p normalisation;
  * the default-start heuristic of the Gauss + exponential model;
  * theta <-> standardised target maps and column statistics.
Pass rounding=False for the same network in plain FP64 (used to pin the
backward pass against finite differences).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

IN, HIDDEN, OUT, OUT_PAD = 256, 512, 5, 32
LAYERS = [(HIDDEN, IN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (OUT_PAD, HIDDEN)]  # (out, in)


def layout():
    """(weight offset, bias offset) per layer in the flat parameter vector."""
    offs, o = [], 0
    for out, inn in LAYERS:
        offs.append((o, o + out * inn))
        o += out * inn + out
    return offs, o


OFFSETS, NPARAMS = layout()


def bf16(x):
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    Ws, bs = [], []
    for (wo, bo), (out, inn) in zip(OFFSETS, LAYERS):
        Ws.append(p[wo:wo + out * inn].reshape(out, inn))
        bs.append(p[bo:bo + out])
    return Ws, bs


def init_params(seed):
    """He-style initial weights (padding rows of the last layer zero)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAMS)
    for (wo, bo), (out, inn) in zip(OFFSETS, LAYERS):
        W = rng.standard_normal((out, inn)) * math.sqrt(2.0 / inn)
        if out == OUT_PAD:
            W *= 0.5
            W[OUT:] = 0.0
        p[wo:wo + out * inn] = W.reshape(-1)
    return p


def forward(params, x, rounding=True):
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    Ws, bs = unpack(params)
    a = r(x)
    cache = {"a": [a], "z": []}
    for l in range(3):
        z = a @ r(Ws[l]).T + bs[l]
        a = r(gelu(z))
        cache["z"].append(z)
        cache["a"].append(a)
    y = a @ r(Ws[3]).T + bs[3]
    return y, cache


def loss_and_grad(params, x, t, rounding=True):
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    B = x.shape[0]
    y, cache = forward(params, x, rounding)
    d = np.zeros_like(y)
    d[:, :OUT] = y[:, :OUT] - t
    loss = float(np.sum(d[:, :OUT] ** 2) / (OUT * B))
    Ws, _ = unpack(params)
    grads = np.zeros(NPARAMS)
    dz = r(2.0 * d / (OUT * B))
    for l in (3, 2, 1, 0):
        (wo, bo), (out, inn) = OFFSETS[l], LAYERS[l]
        grads[wo:wo + out * inn] = (dz.T @ cache["a"][l]).reshape(-1)
        grads[bo:bo + out] = dz.sum(axis=0)
        if l > 0:
            da = dz @ r(Ws[l])
            dz = r(da * gelu_prime(cache["z"][l - 1]))
    return loss, grads, y


def adamw_step(params, m, v, g, step, lr, wd):
    m = 0.9 * m + 0.1 * g
    v = 0.999 * v + 0.001 * g * g
    mh = m / (1 - 0.9 ** step)
    vh = v / (1 - 0.999 ** step)
    params = params - lr * (mh / (np.sqrt(vh) + 1e-8) + wd * params)
    return params, m, v


def rebin_lognorm(counts_concat, offsets, mean, std):
    out = np.zeros((len(offsets) - 1, IN))
    for b in range(len(offsets) - 1):
        c = np.asarray(counts_concat[offsets[b]:offsets[b + 1]], dtype=np.float64)
        nb = c.size
        j = ((2 * np.arange(nb) + 1) * IN) // (2 * nb)  # coarse bin of each fine bin centre
        sums = np.bincount(j, weights=c, minlength=IN)
        k = np.bincount(j, minlength=IN).astype(np.float64)
        v = np.where(k > 0, np.log1p(sums / np.where(k > 0, k, 1.0)), 0.0)
        out[b] = (v - mean) / std
    return out


def default_starts(counts_concat, offsets, ranges, t_shift=0.0, t_scale=1.0):
    B = len(offsets) - 1
    th = np.zeros((B, 5))
    for b in range(B):
        c = np.asarray(counts_concat[offsets[b]:offsets[b + 1]], dtype=np.float64)
        nb = c.size
        lo, hi = ranges[b]
        h = (hi - lo) / nb
        ne = max(nb // 25, 1)
        bk0 = max(c[:ne].sum() / ne, 1.0)
        bk1 = max(c[nb - ne:].sum() / ne, 1.0)
        c0, c1 = 0.5 * ne, nb - 0.5 * ne
        W = max(nb // 256, 1)
        wlen = 2 * W + 1

        lb0 = math.log(bk0)
        dlb = math.log(bk1) - lb0

        def excess(i):
            # window sum minus the exponential background through the edge means
            s = c[i - W:i + W + 1].sum()
            bg = math.exp(lb0 + dlb * ((i + 0.5 - c0) / (c1 - c0)))
            return int(np.rint(s - wlen * bg))

        best, imax = None, nb // 2
        for i in range(W, nb - W):
            e = excess(i)
            if best is None or e > best:
                best, imax = e, i
        if best is None:
            best, imax = 0, nb // 2
        bounds = []
        for d in (-1, 1):
            i = imax
            while True:
                nx = i + d
                if nx < W or nx >= nb - W:
                    break
                if 2 * excess(nx) < best:
                    break
                i = nx
            bounds.append(i)
        rng_ = hi - lo
        fwhm = (bounds[1] - bounds[0] + 1) * h
        s = min(max(fwhm / 2.3548200450309493, 0.005 * rng_), 0.1 * rng_)
        A = max(best / wlen, 1.0)
        m = lo + (imax + 0.5) * h
        t0 = (lo + c0 * h - t_shift) / t_scale
        t1 = (lo + c1 * h - t_shift) / t_scale
        b1 = math.log(bk1 / bk0) / (t1 - t0)
        b0 = math.log(bk0) - b1 * t0
        th[b] = (A, m, s, b0, b1)
    return th


def theta_to_target(theta, mean, std):
    th = np.asarray(theta, dtype=np.float64)
    raw = np.stack([th[:, 1], np.log(np.abs(th[:, 2])), np.log(np.abs(th[:, 0])), th[:, 3], th[:, 4]],
                   axis=1)
    return (raw - mean) / std


def target_to_theta(y, mean, std):
    v = np.asarray(y, dtype=np.float64)[:, :OUT] * std + mean
    return np.stack([np.exp(v[:, 2]), v[:, 0], np.exp(v[:, 1]), v[:, 3], v[:, 4]], axis=1)


def column_stats(x):
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean(axis=0)
    sd = np.sqrt(np.maximum((x * x).mean(axis=0) - mu * mu, 0.0))
    return mu, np.where(sd > 0, sd, 1.0)

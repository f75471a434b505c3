"""Learned initialiser on the GPU against the numpy oracle (oracle/mlp.py).

The kernels and the oracle round to BF16 at the same points; the kernels sum
products in FP32 (MFMA), the oracle in FP64, so a value near a BF16 rounding
boundary can round differently, and such a flip then propagates through the
later layers.  Two gates:
  * element by element, layer by layer: each layer's outputs are recomputed
    in FP64 from the GPU's own stored inputs of that layer (read from the
    workspace), so the only difference left is the FP32 accumulation.  Every
    FP32 result must lie within (K + 2) 2^-24 sum_k |a_k||w_k| of the FP64
    value (K the length of the dot product: the standard bound for a
    recursively summed dot product), and every BF16 result must equal the
    FP64 value rounded to BF16 or sit one BF16 spacing from it, the latter
    for under 1% of the elements (a rounding boundary within the FP32 error);
  * end to end against the oracle's own forward and backward passes,
    norm-wise per layer (relative Frobenius error), where the flips of the
    earlier layers are part of the difference.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def _dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def rel_fro(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


U32 = 2.0 ** -24  # unit roundoff of FP32


def bf16_values(t):
    """A device int16 tensor of BF16 bit patterns as FP64 values."""
    u = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def bf16_spacing(v):
    """Distance from |v| to the next BF16 value up (8 significant bits)."""
    e = np.floor(np.log2(np.maximum(np.abs(v), 2.0 ** -126)))
    return 2.0 ** (e - 7)


def check_fp32_dot(gpu, ref, scale, K, what):
    """FP32 accumulation of K products (plus a bias) against FP64."""
    bound = (K + 2) * U32 * scale + 1e-30
    err = np.abs(np.asarray(gpu, dtype=np.float64) - ref)
    assert np.all(err <= bound), (what, float(np.max(err / bound)))


def check_bf16_rounding(gpu, exact, slack, what, max_flip=0.01):
    """gpu: BF16 results; exact: the FP64 value they round; slack: the error
    bound of the value the GPU rounded (FP32 sums and elementary functions).
    Each result must be the BF16 rounding of some value within `slack` of
    exact: |gpu - exact| <= half a BF16 spacing + slack.  Results that differ
    from bf16(exact) (a rounding boundary within the slack) must be rare."""
    from oracle import mlp as om
    sp = np.maximum(bf16_spacing(exact), bf16_spacing(gpu))
    err = np.abs(gpu - exact)
    bound = 0.5 * sp + slack + 1e-38
    assert np.all(err <= bound), (what, float(np.max(err / bound)))
    flipped = gpu != om.bf16(exact)
    assert flipped.mean() <= max_flip, (what, float(flipped.mean()))


def check_forward_layers(views, p, x, B, train):
    """Each layer of the forward pass against FP64 from the GPU's own inputs."""
    from oracle import mlp as om
    Ws, bs = om.unpack(p)
    a = [bf16_values(views["a%d" % l]) for l in range(4)]
    np.testing.assert_array_equal(a[0], om.bf16(x))  # the input cast is exact
    for l in range(3):
        W = om.bf16(Ws[l])
        b32 = bs[l].astype(np.float32).astype(np.float64)
        zref = a[l] @ W.T + b32
        scale = np.abs(a[l]) @ np.abs(W).T + np.abs(b32)
        K = a[l].shape[1]
        if train:
            z = views["z%d" % (l + 1)].cpu().numpy().astype(np.float64)
            check_fp32_dot(z, zref, scale, K, "z%d" % (l + 1))
        # FP32 sum error through |GELU'| <= 1.13, plus the FP32 GELU's own
        # error, absolute ~|z| u where 1 + erf(z/sqrt2) cancels (z < 0)
        slack = (K + 2) * U32 * scale * 1.13 + 4 * U32 * (np.abs(zref) + np.abs(om.gelu(zref)))
        check_bf16_rounding(a[l + 1], om.gelu(zref), slack, "a%d" % (l + 1))
    W = om.bf16(Ws[3])
    b32 = bs[3].astype(np.float32).astype(np.float64)
    yref = a[3] @ W.T + b32
    scale = np.abs(a[3]) @ np.abs(W).T + np.abs(b32)
    return a, yref, scale


@pytest.mark.parametrize("batch", [64, 192])
def test_forward_layers_elementwise(hf, batch):
    """Inference: every hidden activation and every output element against
    FP64 recomputed from the GPU's own layer inputs."""
    import torch
    from oracle import mlp as om
    rng = np.random.default_rng(100 + batch)
    p = om.init_params(7)
    x = rng.standard_normal((batch, om.IN))
    ws = hf.mlp_workspace(batch, "cuda")
    y = hf.mlp_forward(_dev(p, torch.float32), _dev(x, torch.float32), workspace=ws)
    torch.cuda.synchronize()
    views = hf.mlp_workspace_views(ws, batch)
    _, yref, scale = check_forward_layers(views, p, x, batch, train=False)
    y = y.cpu().numpy().astype(np.float64)
    check_fp32_dot(y[:, :5], yref[:, :5], scale[:, :5], om.HIDDEN, "y")
    np.testing.assert_array_equal(y[:, 5:], 0.0)


def test_train_step_layers_elementwise(hf):
    """One training step, every stored value and every gradient element
    against FP64 recomputed from the GPU's own inputs of that step."""
    import torch
    from oracle import mlp as om
    rng = np.random.default_rng(12)
    B = 128
    p = om.init_params(8)
    x = rng.standard_normal((B, om.IN))
    t = rng.standard_normal((B, om.OUT))
    P = _dev(p, torch.float32)
    m, v, g = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = hf.mlp_workspace(B, "cuda")
    hf.mlp_train_step(P, m, v, 1, 1e-3, 1e-4, _dev(x, torch.float32), _dev(t, torch.float32), g,
                      loss, ws)
    torch.cuda.synchronize()
    views = hf.mlp_workspace_views(ws, B)
    a, yref, yscale = check_forward_layers(views, p, x, B, train=True)
    y = views["y"].cpu().numpy().astype(np.float64)
    check_fp32_dot(y[:, :5], yref[:, :5], yscale[:, :5], om.HIDDEN, "y")
    # output adjoint: dz4 = bf16(2 (y - t) / (5 B)) from the GPU's own y
    t32 = t.astype(np.float32).astype(np.float64)
    d4 = 2.0 * (y[:, :5] - t32) / (5 * B)
    dz = {4: bf16_values(views["dz4"])}
    check_bf16_rounding(dz[4][:, :5], d4, 4 * U32 * (np.abs(y[:, :5]) + np.abs(t32)) * 2.0 / (5 * B),
                        "dz4")
    np.testing.assert_array_equal(dz[4][:, 5:], 0.0)
    Ws, _ = om.unpack(p)
    gg = g.cpu().numpy().astype(np.float64)
    for l in (3, 2, 1, 0):
        (wo, bo), (out, inn) = om.OFFSETS[l], om.LAYERS[l]
        rows = om.OUT if out == om.OUT_PAD else out
        d = dz[l + 1][:, :rows]
        # weight gradient dW = dz^T a and bias gradient sum_b dz, over B rows
        gw = gg[wo:wo + out * inn].reshape(out, inn)
        check_fp32_dot(gw[:rows], d.T @ a[l], np.abs(d).T @ np.abs(a[l]), B, "dW%d" % l)
        np.testing.assert_array_equal(gw[rows:], 0.0)
        check_fp32_dot(gg[bo:bo + rows], d.sum(axis=0), np.abs(d).sum(axis=0), B, "db%d" % l)
        if l > 0:
            # dz_l = bf16(GELU'(z_l) * (dz_{l+1} W_l)) from the GPU's dz_{l+1}, z_l
            W = om.bf16(Ws[l])[:rows]
            z = views["z%d" % l].cpu().numpy().astype(np.float64)
            gp = om.gelu_prime(z)
            C = d @ W
            exact = C * gp
            # FP32 sum error times GELU', plus GELU''s own FP32 error (a few
            # u absolute) times the sum, plus the product's rounding
            slack = (rows + 2) * U32 * (np.abs(d) @ np.abs(W)) * (np.abs(gp) + 8 * U32) + \
                8 * U32 * np.abs(C) + 4 * U32 * np.abs(exact)
            dz[l] = bf16_values(views["dz%d" % l])
            check_bf16_rounding(dz[l], exact, slack, "dz%d" % l)


@pytest.mark.parametrize("batch", [64, 192])
def test_forward_matches_oracle(hf, batch):
    import torch
    from oracle import mlp as om
    rng = np.random.default_rng(batch)
    p = om.init_params(5)
    x = rng.standard_normal((batch, om.IN))
    y_ref, _ = om.forward(p, x)
    y = hf.mlp_forward(_dev(p, torch.float32), _dev(x, torch.float32))
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    assert rel_fro(y[:, :5], y_ref[:, :5]) < 2e-3
    np.testing.assert_array_equal(y[:, 5:], 0.0)


def test_train_step_matches_oracle(hf):
    import torch
    from oracle import mlp as om
    rng = np.random.default_rng(11)
    B = 128
    p = om.init_params(6)
    x = rng.standard_normal((B, om.IN))
    t = rng.standard_normal((B, om.OUT))
    loss_ref, g_ref, _ = om.loss_and_grad(p, x, t)
    P = _dev(p, torch.float32)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    g = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ws = hf.mlp_workspace(B, "cuda")
    hf.mlp_train_step(P, m, v, 1, 1e-3, 1e-4, _dev(x, torch.float32), _dev(t, torch.float32), g, loss, ws)
    torch.cuda.synchronize()
    assert loss.item() == pytest.approx(loss_ref, rel=2e-3)
    gg = g.cpu().numpy().astype(np.float64)
    for l, ((wo, bo), (out, inn)) in enumerate(zip(om.OFFSETS, om.LAYERS)):
        rows = om.OUT if out == om.OUT_PAD else out
        gw = gg[wo:wo + out * inn].reshape(out, inn)[:rows]
        rw = g_ref[wo:wo + out * inn].reshape(out, inn)[:rows]
        assert rel_fro(gw, rw) < 2e-2, l
        assert rel_fro(gg[bo:bo + rows], g_ref[bo:bo + rows]) < 2e-2, l
        np.testing.assert_array_equal(gg[wo + rows * inn:wo + out * inn], 0.0)
    # AdamW applied to the kernel's own gradient, in FP64
    p1, _, _ = om.adamw_step(p, np.zeros_like(p), np.zeros_like(p), gg, 1, 1e-3, 1e-4)
    np.testing.assert_allclose(P.cpu().numpy(), p1, rtol=1e-5, atol=1e-7)


def test_rebin_and_starts_match_oracle(hf):
    import torch
    from oracle import mlp as om
    c = datagen.batch_case(seed=21, B=24, lo_bins=100, hi_bins=20000)
    counts = torch.from_numpy(c["counts"].view(np.int32)).cuda()
    x = hf.rebin_lognorm(counts, c["offsets"], 1.5, 2.0)
    th0 = hf.default_starts(counts, c["offsets"], c["ranges"], hf.Model(hf.GAUSS_EXP, 1, -1))
    torch.cuda.synchronize()
    np.testing.assert_allclose(x.cpu().numpy(), om.rebin_lognorm(c["counts"], c["offsets"], 1.5, 2.0),
                               rtol=2e-6, atol=1e-6)
    ref = om.default_starts(c["counts"], c["offsets"], c["ranges"])
    np.testing.assert_allclose(th0.cpu().numpy(), ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("dtype", ["u32", "f64"])
def test_default_starts_edge_sizes(hf, dtype):
    """Window range empty (1, 2 bins) or one position (3), sizes around the
    256-bin window step, a flat histogram (every excess ties), a peak at the
    edge, and the largest batch size; integer counts also as FP64."""
    import torch
    from oracle import mlp as om
    rng = np.random.default_rng(77)
    hists = [np.array([5.0]), np.array([3.0, 9.0]), np.array([1.0, 7.0, 2.0]),
             np.full(300, 40.0), rng.poisson(20, 255).astype(float), rng.poisson(20, 256).astype(float),
             rng.poisson(20, 257).astype(float), rng.poisson(20, 511).astype(float)]
    for nb, m in ((65536, 0.37), (4096, 0.002), (4096, 0.999), (20000, 0.5)):
        x = (np.arange(nb) + 0.5) / nb
        hists.append(rng.poisson(300 * np.exp(-0.5 * ((x - m) / 0.02) ** 2) + 50).astype(float))
    off = np.zeros(len(hists) + 1, dtype=np.int64)
    off[1:] = np.cumsum([h.size for h in hists])
    cat = np.concatenate(hists)
    rg = np.tile([0.0, 1.0], (len(hists), 1))
    if dtype == "u32":
        counts = torch.from_numpy(cat.astype(np.uint32).view(np.int32)).cuda()
    else:
        counts = torch.from_numpy(cat).cuda()
    th0 = hf.default_starts(counts, off, rg, hf.Model(hf.GAUSS_EXP, 1, -1))
    torch.cuda.synchronize()
    ref = om.default_starts(cat, off, rg)
    np.testing.assert_allclose(th0.cpu().numpy(), ref, rtol=1e-10, atol=1e-12)


def test_target_maps_and_stats(hf):
    import torch
    from oracle import mlp as om
    rng = np.random.default_rng(3)
    th = np.stack([np.exp(rng.uniform(4, 9, 300)), rng.uniform(0, 1, 300), rng.uniform(0.01, 0.05, 300),
                   rng.uniform(2, 7, 300), rng.uniform(-3, 3, 300)], axis=1)
    raw = hf.theta_to_target(_dev(th, torch.float64), torch.zeros(5, device="cuda"),
                             torch.ones(5, device="cuda"))
    mean, std = hf.column_stats(raw)
    t = hf.theta_to_target(_dev(th, torch.float64), mean, std)
    y = torch.zeros(300, 32, device="cuda")
    y[:, :5] = t
    back = hf.target_to_theta(y, mean, std)
    torch.cuda.synchronize()
    mu, sd = om.column_stats(om.theta_to_target(th, 0.0, 1.0))
    np.testing.assert_allclose(mean.cpu().numpy(), mu, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(std.cpu().numpy(), sd, rtol=1e-6)
    # the target is FP32: a parameter near zero keeps an absolute error of
    # about half an FP32 ulp of the standardised value times the column std
    t_np = t.cpu().numpy().astype(np.float64)
    atol = 2.0 ** -23 * (np.abs(t_np).max(axis=0) * std.cpu().numpy() + np.abs(mean.cpu().numpy()))
    np.testing.assert_allclose(back.cpu().numpy(), th, rtol=2e-6, atol=float(atol.max()))


def test_training_reduces_loss(hf):
    import torch
    from paper_2203_06139_amd.learned_init import LearnedInit
    li = LearnedInit("cuda", seed=1, batch=256)
    counts, off, rg, theta = datagen.batch_case_device(101, 2048, 4096, "cuda")
    li.x = hf.rebin_lognorm(counts, off, 3.0, 1.5)
    raw = hf.theta_to_target(theta.cuda(), torch.zeros(5, device="cuda"), torch.ones(5, device="cuda"))
    li.t_mean, li.t_std = hf.column_stats(raw)
    li.t = hf.theta_to_target(theta.cuda(), li.t_mean, li.t_std)
    hist = li.train(epochs=6, lr=2e-3, log=lambda *a: None)
    assert hist[-1] < 0.5 * hist[0], hist


@pytest.mark.slow
def test_learned_init_beats_plain_starts(hf):
    """Train on 524,288 plain fits of 4096-bin histograms, then fit an uneven
    4096-histogram batch (256..65536 bins, seeds disjoint from training) from
    the learned start with plain-start fallback.  The plain fit judges: a
    learned fit agrees when both converged and |NLL_learned - NLL_plain| <
    1e-6; a fit that reached a different minimum, lower or higher, is a
    disagreement.  More than 98% of the histograms must agree, the learned
    fits need fewer iterations on average, and the learned path (rebin,
    network, fits, refits) takes less time than the plain one (default
    starts, fits)."""
    import torch
    from paper_2203_06139_amd.learned_init import FitSet, LearnedInit, plain_fit, timed
    li = LearnedInit("cuda", seed=2, batch=1024)
    kept = li.build_training_set(524288, seed=1000, log=lambda *a: None)
    assert kept > 500000
    li.train(epochs=8, lr=1e-3, log=lambda *a: None)
    c = datagen.batch_case(seed=7)
    fs = FitSet(torch.from_numpy(c["counts"].view(np.int32)).cuda(),
                torch.as_tensor(c["offsets"]).cuda(), torch.as_tensor(c["ranges"]).cuda())
    plain_fit(fs)
    li.fit(fs)  # warm-up of both paths
    (_, plain), t_plain = timed(lambda: plain_fit(fs))
    (learned, nfb), t_learned = timed(lambda: li.fit(fs))
    B = plain.status.numel()
    both = (plain.status == 0) & (learned.status == 0)
    dn = learned.nll - plain.nll
    agree = both & (dn.abs() < 1e-6)
    lower = both & (dn <= -1e-6)
    higher = both & (dn >= 1e-6)
    summary = dict(agree=int(agree.sum()), lower=int(lower.sum()), higher=int(higher.sum()),
                   not_both=int(B - both.sum()), fallbacks=nfb)
    assert agree.float().mean().item() > 0.98, summary
    it_p = plain.iters.float().mean().item()
    it_l = learned.iters.float().mean().item()
    assert it_l < it_p, (it_l, it_p, summary)
    assert t_learned < t_plain, (t_learned, t_plain, summary)

"""Learned initialiser on the GPU against the numpy oracle (oracle/mlp.py).

The kernels and the oracle round to BF16 at the same points; the kernels sum
products in FP32 (MFMA), the oracle in FP64, so a value near a BF16 rounding
boundary can round differently.  Comparisons are therefore norm-wise per
layer (relative Frobenius error) with a bound on the largest element error.
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
    the learned start with plain-start fallback.  Where both converge, the
    learned fit's NLL is within 1e-6 of the plain fit's or below it for more
    than 99% of the histograms, it needs fewer iterations on average, and
    the learned path (rebin, network, fits, refits) takes less time than the
    plain one (default starts, fits)."""
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
    both = (plain.status == 0) & (learned.status == 0)
    assert both.float().mean().item() > 0.97
    ok = (learned.nll - plain.nll)[both] < 1e-6
    assert ok.float().mean().item() > 0.99, (learned.nll - plain.nll)[both].max().item()
    it_p = plain.iters.float().mean().item()
    it_l = learned.iters.float().mean().item()
    assert it_l < it_p, (it_l, it_p, nfb)
    assert t_learned < t_plain, (t_learned, t_plain, nfb)

"""GPU fits (fit_batch) against the oracle's BFGS on the same starts.

Agreement criterion: both fits converge and |NLL_gpu - NLL_oracle| < 1e-6
(absolute, saturated Poisson scale, FP64 re-evaluation); the fitted
parameters then agree to within a small fraction of their scale.
"""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def orc_model(orc, spec):
    return orc.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"])


def to_dev_counts(counts):
    import torch
    return torch.from_numpy(np.ascontiguousarray(counts).view(np.int32)).cuda()


def run_fit(hf, spec, counts, offsets, ranges, theta0, **kw):
    import torch
    r = hf.fit_batch(to_dev_counts(counts), torch.as_tensor(offsets), torch.as_tensor(ranges),
                     hf.Model.from_spec(spec), torch.as_tensor(theta0), **kw)
    torch.cuda.synchronize()
    return (r.theta.cpu().numpy(), r.nll.cpu().numpy(), r.status.cpu().numpy(),
            r.iters.cpu().numpy(), r.nevals.cpu().numpy())


@pytest.mark.parametrize("hinit", [0, 1])
@pytest.mark.parametrize("obj", [2, 0])
def test_single_fit_10k_bins(hf, orc, obj, hinit):
    c = datagen.single_fit_case()
    th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], [0, c["counts"].size],
                                  [c["range"]], c["theta0"][None, :], objective=obj,
                                  hessian_init=hinit)
    ref = orc.fit(orc_model(orc, c["spec"]), obj, c["counts"], c["theta0"], c["range"],
                  hessian_init=hinit)
    assert ref.status == 0 and st[0] == 0, (ref, st)
    assert abs(nll[0] - ref.nll) < 1e-6, (nll[0], ref.nll)
    np.testing.assert_allclose(th[0], ref.theta, rtol=1e-5, atol=1e-6)
    assert it[0] >= 1 and ne[0] >= it[0]
    assert abs(int(it[0]) - ref.iters) <= max(2, ref.iters // 5), (it[0], ref.iters)


def _subset(B, seed=3):
    c = datagen.batch_case(seed=seed, B=B, lo_bins=256, hi_bins=16384)
    rng = np.random.default_rng(seed + 77)
    th0 = c["theta_true"].copy()
    th0[:, 0] *= 1 + 0.05 * rng.standard_normal(B)
    th0[:, 1] += 0.3 * th0[:, 2] * rng.standard_normal(B)
    th0[:, 2] *= 1 + 0.05 * rng.standard_normal(B)
    th0[:, 3] += 0.05 * rng.standard_normal(B)
    th0[:, 4] += 0.05 * rng.standard_normal(B)
    return c, th0


@pytest.mark.parametrize("hinit", [0, 1])
@pytest.mark.parametrize("prec", [0, 1])
def test_batched_fits_match_oracle(hf, orc, prec, hinit):
    c, th0 = _subset(96)
    kw = dict(objective=2, precision=prec, polish_edm=1e-3 if prec else 0.0, hessian_init=hinit)
    th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], th0, **kw)
    rth, rnll, rst, rit, rne = orc.fit_many(orc_model(orc, c["spec"]), 2, c["counts"],
                                           c["offsets"], c["ranges"], th0, nthreads=8,
                                           hessian_init=hinit)
    both = (st == 0) & (rst == 0)
    assert both.mean() > 0.9, (st, rst)
    dn = np.abs(nll - rnll)[both]
    assert np.all(dn < 1e-6), dn.max()
    scale = np.maximum(np.abs(rth[both]), 1e-3)
    assert np.all(np.abs(th[both] - rth[both]) <= 1e-3 * scale)


@pytest.mark.parametrize("obj", [2, 0, 1])
def test_first_fisher_step_matches_oracle(hf, orc, obj):
    """One iteration from the same start: the step is -H0 g with H0 the
    inverse expected Hessian, so theta after it checks the device's F, its
    scaled Cholesky inverse and the first line-search acceptance against
    the oracle.  The two F differ only in summation order."""
    c, th0 = _subset(24, seed=5)
    M = orc_model(orc, c["spec"])
    th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], th0,
                                  objective=obj, max_iter=1, fixed_iters=True, hessian_init=1)
    for b in range(24):
        seg = c["counts"][c["offsets"][b]:c["offsets"][b + 1]].astype(np.float64)
        ref = orc.fit(M, obj, seg, th0[b], c["ranges"][b], max_iter=1, fixed_iters=True,
                      hessian_init=1)
        assert it[b] == ref.iters and ne[b] == ref.nevals, (b, it[b], ref.iters, ne[b], ref.nevals)
        scale = np.maximum(np.abs(th0[b] - ref.theta), 1e-12 * np.maximum(np.abs(ref.theta), 1.0))
        assert np.all(np.abs(th[b] - ref.theta) <= 1e-6 * scale + 1e-12 * np.abs(ref.theta)), b


def test_fisher_start_cuts_iterations(hf):
    """Default-start fits of a batch: the Fisher start reaches the same
    minima as the identity start in far fewer iterations."""
    import torch
    c = datagen.batch_case(seed=41, B=256, lo_bins=256, hi_bins=16384)
    counts = to_dev_counts(c["counts"])
    off = torch.as_tensor(c["offsets"]).cuda()
    rg = torch.as_tensor(c["ranges"]).cuda()
    m = hf.Model.from_spec(c["spec"])
    t0 = hf.default_starts(counts, off, rg, m)
    r0 = hf.fit_batch(counts, off, rg, m, t0, hessian_init=hf.IDENTITY)
    r1 = hf.fit_batch(counts, off, rg, m, t0, hessian_init=hf.FISHER)
    torch.cuda.synchronize()
    both = (r0.status == 0) & (r1.status == 0)
    assert both.float().mean().item() > 0.95
    dn = (r0.nll - r1.nll).abs()[both]
    assert (dn < 1e-6).float().mean().item() > 0.95
    assert r1.iters.float().mean().item() < 0.5 * r0.iters.float().mean().item()


@pytest.mark.parametrize("waves", [False, True])
def test_bad_histograms_and_status_codes(hf, waves):
    """Status codes of fit_batch, with one workgroup per histogram and with
    every histogram (empty ones included) fitted by a wave of its own."""
    c, th0 = _subset(4)
    m = hf.Model.from_spec(c["spec"])
    wave_bins = hf.fit_max_wave_bins(m, hf.POISSON, 256) if waves else 0
    assert wave_bins == 0 or wave_bins >= max(np.diff(c["offsets"]))
    off = c["offsets"].copy()
    off[2] = off[1]  # histogram 1 empty
    ranges = c["ranges"].copy()
    ranges[3] = (1.0, 1.0)  # histogram 3: empty range
    try:
        hf.fit_set_wave_bins(wave_bins)
        th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], off, ranges, th0)
        assert st[1] == hf.FIT_BADHIST and st[3] == hf.FIT_BADHIST
        np.testing.assert_array_equal(th[1], th0[1])
        assert st[0] == hf.FIT_CONVERGED
        th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], th0,
                                      max_iter=1)
        assert np.all(st == hf.FIT_MAXITER) and np.all(it == 1)
    finally:
        hf.fit_set_wave_bins(0)


def test_fit_batch_repeatable_and_graph_replay(hf):
    import torch
    c, th0 = _subset(64, seed=11)
    counts = to_dev_counts(c["counts"])
    off = torch.as_tensor(c["offsets"]).cuda()
    rg = torch.as_tensor(c["ranges"]).cuda()
    t0 = torch.as_tensor(th0).cuda()
    m = hf.Model.from_spec(c["spec"])
    eager = hf.fit_batch(counts, off, rg, m, t0, precision=1, polish_edm=1e-3)
    torch.cuda.synchronize()
    ref = (eager.theta.clone(), eager.nll.clone(), eager.status.clone())
    again = hf.fit_batch(counts, off, rg, m, t0, precision=1, polish_edm=1e-3)
    torch.cuda.synchronize()
    assert torch.equal(again.theta, ref[0]) and torch.equal(again.nll, ref[1])
    # capture into a graph and replay, with eager work between replays
    out = hf.FitBatchResult(torch.empty_like(ref[0]), torch.empty_like(ref[1]),
                            torch.empty_like(ref[2]), torch.empty_like(ref[2]),
                            torch.empty_like(ref[2]))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        hf.fit_batch(counts, off, rg, m, t0, precision=1, polish_edm=1e-3, out=out)  # warm-up
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            hf.fit_batch(counts, off, rg, m, t0, precision=1, polish_edm=1e-3, out=out)
    torch.cuda.synchronize()
    for _ in range(3):
        out.theta.zero_()
        out.nll.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.theta, ref[0]) and torch.equal(out.nll, ref[1])
        x = torch.randn(1000, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        del x
    # a larger uncaptured batch on the capturing stream's context must not
    # move the scratch the graph holds: replays still give the eager result
    big, bth0 = _subset(200, seed=12)
    with torch.cuda.stream(s):
        hf.fit_batch(to_dev_counts(big["counts"]), torch.as_tensor(big["offsets"]).cuda(),
                     torch.as_tensor(big["ranges"]).cuda(), m, torch.as_tensor(bth0).cuda(),
                     precision=1, polish_edm=1e-3)
    torch.cuda.synchronize()
    for _ in range(2):
        out.theta.zero_()
        out.nll.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.theta, ref[0]) and torch.equal(out.nll, ref[1])


def test_calls_on_two_streams_use_separate_scratch(hf):
    """Objective calls on two streams, each serialised on its own stream but
    free to overlap with the other, give the single-stream results: every
    stream has its own context, so the block partials and completion ticket
    are never shared between overlapping launches."""
    import torch
    spec = datagen.model_spec(1, 2, 3, 50.0, 50.0)
    th = [700.0, 30.0, 4.0, 400.0, 62.0, 6.0, 100.0, -20.0, 10.0, 5.0]
    cases = [datagen.random_1d_case(spec, 2_000_003 + k, 0.0, 100.0, th, seed=40 + k)
             for k in range(2)]
    m = hf.Model.from_spec(spec)
    hists = [hf.make_hist(c["counts"], (0.0, 100.0)) for c in cases]
    thetas = [torch.as_tensor(c["theta_eval"], dtype=torch.float64, device="cuda")
              for c in cases]
    ref = []
    for h, t in zip(hists, thetas):
        n, g_, _ = hf.nll_grad(h, m, t)
        ref.append((n.clone(), g_.clone()))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    outs = [[], []]
    for rep in range(8):
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                outs[k].append(hf.nll_grad(hists[k], m, thetas[k])[:2])
    torch.cuda.synchronize()
    for k in range(2):
        for n, g_ in outs[k]:
            assert torch.equal(n, ref[k][0]) and torch.equal(g_, ref[k][1]), k


def test_strided_and_mistyped_tensors_are_refused(hf):
    """The kernels read plain pointers, so the binding refuses tensors whose
    memory is not laid out as the call reads it."""
    import torch
    m = hf.Model(hf.GAUSS_POLY, 1, 1)
    th = [10.0, 0.5, 0.1, 1.0, 0.0]
    c2 = torch.ones(64, 64, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="contiguous"):
        hf.nll_eval(hf.Hist(c2.t(), (0.0, 1.0), (0.0, 1.0)), hf.Model(hf.GAUSS2D),
                    [1.0, 0.5, 0.5, 0.1, 0.1, 0.0, 1.0])
    c = torch.ones(128, dtype=torch.int32, device="cuda")
    w = torch.ones(256, dtype=torch.float32, device="cuda")[::2]
    with pytest.raises(ValueError):
        hf.nll_grad(hf.Hist(c, (0.0, 1.0), weights=w), m, th)
    with pytest.raises(ValueError):
        hf.nll_grad(hf.Hist(c, (0.0, 1.0), weights=torch.ones(128, device="cuda",
                                                               dtype=torch.float64)), m, th)
    with pytest.raises(ValueError):
        hf.nll_grad(hf.Hist(c, (0.0, 1.0)), m, th,
                    grad_out=torch.empty(5, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        hf.nll_grad(hf.Hist(c, (0.0, 1.0)), m, th, want_grad_w=True,
                    grad_w_out=torch.empty(256, dtype=torch.float32, device="cuda")[::2])


def test_launch_shape_does_not_change_results(hf, orc):
    """Every workgroup size, workgroups per CU and LDS cache setting fits the
    same batch to the same minima (summation order aside), and matches the
    oracle; out-of-range settings are refused without touching the state."""
    c, th0 = _subset(48, seed=13)
    m = hf.Model.from_spec(c["spec"])
    rth, rnll, rst, _, _ = orc.fit_many(orc_model(orc, c["spec"]), 2, c["counts"], c["offsets"],
                                        c["ranges"], th0, nthreads=8, hessian_init=1)
    try:
        for blk, wg in ((256, 1), (512, 1), (512, 4), (256, 8)):
            cap = hf.fit_max_cache_bins(m, hf.POISSON, blk)
            assert cap > 4096
            for cb in (0, cap):
                hf.fit_set_tuning(wg, cb, blk)
                assert hf.fit_get_tuning() == (wg, cb, blk)
                th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], c["offsets"],
                                              c["ranges"], th0, objective=2)
                both = (st == 0) & (rst == 0)
                assert both.mean() > 0.9, (blk, wg, cb)
                assert np.all(np.abs(nll - rnll)[both] < 1e-6), (blk, wg, cb)
        for bad in ((0, 0, 256), (2, -1, 256), (2, 0, 384)):
            with pytest.raises(hf.HistfitError):
                hf.fit_set_tuning(*bad)
        assert hf.fit_get_tuning() == (8, hf.fit_max_cache_bins(m, hf.POISSON, 256), 256)
        hf.fit_set_tuning(2, hf.fit_max_cache_bins(m, hf.POISSON, 512) + 1, 512)
        with pytest.raises(hf.HistfitError):
            run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], th0)
    finally:
        hf.fit_set_tuning(2, 0, 256)


def test_autotuner_picks_an_agreeing_shape(hf, tmp_path, monkeypatch):
    import torch
    from paper_2203_06139_amd.autotune import tune_fit
    monkeypatch.setenv("HF_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    c, th0 = _subset(64, seed=17)
    counts = to_dev_counts(c["counts"])
    off = torch.as_tensor(c["offsets"]).cuda()
    rg = torch.as_tensor(c["ranges"]).cuda()
    m = hf.Model.from_spec(c["spec"])
    try:
        best, results = tune_fit(counts, off, rg, m, torch.as_tensor(th0).cuda(), sample=64)
        assert best["agree"] and len(results) > 40
        assert hf.fit_get_tuning() == (best["wg_per_cu"], best["cache_bins"], best["block_size"])
        assert best["ms"] == min(r["ms"] for r in results if r["agree"])
        hf.fit_set_tuning(2, 0, 256)
        again, none = tune_fit(counts, off, rg, m, torch.as_tensor(th0).cuda(), sample=64)
        assert none == [] and again == best  # from the cache file
        assert hf.fit_get_tuning() == (best["wg_per_cu"], best["cache_bins"], best["block_size"])
    finally:
        hf.fit_set_tuning(2, 0, 256)


@pytest.mark.parametrize("K", [1, 3])
def test_finite_difference_fits_reach_the_adjoint_minima(hf, orc, K):
    """Central-difference gradients (the comparison the paper draws) lead the
    same fitter to the oracle's minima; every gradient costs 2 nf value
    sweeps, and FP32 bins are refused for it."""
    c = datagen.kgauss_batch_case(K, seed=9, B=24, nbins=4000)
    P = 3 * K + 2
    kw = dict(objective=2, precision=0)
    ad = run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], c["theta0"],
                 gradient=hf.ADJOINT, **kw)
    fd = run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], c["theta0"],
                 gradient=hf.FINITE_DIFF, **kw)
    rth, rnll, rst, _, _ = orc.fit_many(orc_model(orc, c["spec"]), 2, c["counts"], c["offsets"],
                                        c["ranges"], c["theta0"], nthreads=8, hessian_init=1)
    both = (ad[2] == 0) & (fd[2] == 0) & (rst == 0)
    assert both.mean() > 0.9, (ad[2], fd[2], rst)
    assert np.all(np.abs(ad[1] - rnll)[both] < 1e-6)
    assert np.all(np.abs(fd[1] - rnll)[both] < 1e-6), np.abs(fd[1] - rnll)[both].max()
    # value sweeps: 1 + 2P at the start, then per iteration the trials + 2P
    assert np.all(fd[4] >= (1 + 2 * P) + fd[3] * (1 + 2 * P))
    with pytest.raises(hf.HistfitError):
        run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], c["theta0"],
                gradient=hf.FINITE_DIFF, objective=2, precision=1)


def _sized_subset(B, seed, lo_bins, hi_bins):
    c = datagen.batch_case(seed=seed, B=B, lo_bins=lo_bins, hi_bins=hi_bins)
    rng = np.random.default_rng(seed + 77)
    th0 = c["theta_true"].copy()
    th0[:, 0] *= 1 + 0.05 * rng.standard_normal(B)
    th0[:, 1] += 0.3 * th0[:, 2] * rng.standard_normal(B)
    th0[:, 2] *= 1 + 0.05 * rng.standard_normal(B)
    th0[:, 3] += 0.05 * rng.standard_normal(B)
    th0[:, 4] += 0.05 * rng.standard_normal(B)
    return c, th0


@pytest.mark.parametrize("blk", [256, 512])
def test_wave_per_small_histogram_matches_oracle(hf, orc, blk):
    """Once the longest-first queue reaches histograms of at most wave_bins
    bins, every wave fits its own (state and counts in an LDS slot of its
    own, wave-level reductions): with it off, at 1024 bins and at the model's
    limit, with and without the workgroup count cache, in FP64 and FP32 bins,
    the fits reach the oracle's minima, and a second call (the queue re-armed
    by the first) gives the same results; a wave_bins above the limit is
    refused."""
    c, th0 = _sized_subset(240, seed=41, lo_bins=64, hi_bins=6000)
    rth, rnll, rst, _, _ = orc.fit_many(orc_model(orc, c["spec"]), 2, c["counts"], c["offsets"],
                                        c["ranges"], th0, nthreads=8, hessian_init=1)
    m = hf.Model.from_spec(c["spec"])
    cap_w = hf.fit_max_wave_bins(m, hf.POISSON, blk)
    cap_c = hf.fit_max_cache_bins(m, hf.POISSON, blk)
    assert cap_w >= 2048
    try:
        for wb in (0, 1024, cap_w):
            for cb in (0, cap_c):
                hf.fit_set_tuning(2, cb, blk)
                hf.fit_set_wave_bins(wb)
                assert hf.fit_get_wave_bins() == wb
                for prec in (0, 1):
                    kw = dict(objective=2, precision=prec, polish_edm=1e-3 if prec else 0.0)
                    th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], c["offsets"],
                                                  c["ranges"], th0, **kw)
                    both = (st == 0) & (rst == 0)
                    assert both.mean() > 0.9, (wb, cb, prec, st)
                    assert np.all(np.abs(nll - rnll)[both] < 1e-6), (wb, cb, prec)
                    again = run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], th0, **kw)
                    for x, y in zip((th, nll, st, it, ne), again):
                        np.testing.assert_array_equal(x, y)
        hf.fit_set_wave_bins(cap_w + 1)
        with pytest.raises(hf.HistfitError):
            run_fit(hf, c["spec"], c["counts"], c["offsets"], c["ranges"], th0)
        with pytest.raises(hf.HistfitError):
            hf.fit_set_wave_bins(-1)
    finally:
        hf.fit_set_wave_bins(0)
        hf.fit_set_tuning(2, 0, 256)


def test_eight_bin_sweep_matches_oracle(hf, orc):
    """512-thread workgroups fit histograms of at least 8 x 512 bins of the
    Gauss + exponential model with 8-bin chunks (several rounds of the
    workgroup and ragged tails of chunks and single bins here): with the
    counts streamed from global memory and read from the LDS cache as
    16-byte vectors, in FP64 and FP32 bins, the fits reach the oracle's
    minima, and a 256-thread launch (4-bin chunks) reaches the same ones."""
    c, th0 = _sized_subset(48, seed=43, lo_bins=4096, hi_bins=40000)
    nb = np.diff(c["offsets"])
    assert nb.min() >= 8 * 512 and np.any(nb % 8 != 0) and np.any(nb > 8 * 512 * 4)
    rth, rnll, rst, _, _ = orc.fit_many(orc_model(orc, c["spec"]), 2, c["counts"], c["offsets"],
                                        c["ranges"], th0, nthreads=8, hessian_init=1)
    m = hf.Model.from_spec(c["spec"])
    try:
        for blk in (512, 256):
            cap_c = hf.fit_max_cache_bins(m, hf.POISSON, blk)
            for cb in (0, cap_c):
                hf.fit_set_tuning(1, cb, blk)
                for prec in (0, 1):
                    kw = dict(objective=2, precision=prec, polish_edm=1e-3 if prec else 0.0)
                    th, nll, st, it, ne = run_fit(hf, c["spec"], c["counts"], c["offsets"],
                                                  c["ranges"], th0, **kw)
                    both = (st == 0) & (rst == 0)
                    assert both.mean() > 0.9, (blk, cb, prec, st, rst)
                    assert np.all(np.abs(nll - rnll)[both] < 1e-6), (blk, cb, prec)
                    scale = np.maximum(np.abs(rth[both]), 1e-3)
                    assert np.all(np.abs(th[both] - rth[both]) <= 1e-3 * scale), (blk, cb, prec)
    finally:
        hf.fit_set_tuning(2, 0, 256)

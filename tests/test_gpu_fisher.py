"""GPU parity of hf_nll_fisher and hf_fisher_covariance against the FP64 oracle.

Fisher matrix: |F_gpu - F_ref|_jk <= 1e-10 sqrt(F_jj F_kk).  Every term
w_i c_i J_ij J_ik has w_i c_i > 0, so by Cauchy-Schwarz sqrt(F_jj F_kk)
bounds sum_i |w_i c_i J_ij J_ik|, the condition scale of the sum.

Covariance: both sides invert in FP64 by different routes (Cholesky of the
unit-diagonal scaling here, LAPACK's LU in the oracle), so an entry may differ
by about kappa * eps relative to sqrt(cov_jj cov_kk), kappa the condition
number of the unit-diagonal matrix; the bound is 1e-13 kappa + 1e-14.
"""
import math

import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu

TOL = 1e-10

CASES_1D = [
    (datagen.model_spec(1, 1, 1, 0.0, 1.0), [300.0, 4.8, 0.7, 20.0, -1.2], (0.0, 10.0)),
    (datagen.model_spec(1, 2, 3, 50.0, 50.0),
     [700.0, 30.0, 4.0, 400.0, 62.0, 6.0, 100.0, -20.0, 10.0, 5.0], (0.0, 100.0)),
    (datagen.model_spec(2, 1, -1, 0.0, 1.0), [500.0, 0.45, 0.05, math.log(200.0), math.log(0.3)],
     (0.0, 1.0)),
    (datagen.model_spec(1, 3, 0, 0.0, 1.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 15.0], (0.0, 10.0)),
    (datagen.model_spec(1, 4, 3, 5.0, 5.0),
     [80.0, 2.0, 0.5, 120.0, 5.0, 0.8, 60.0, 7.5, 0.4, 50.0, 8.8, 0.3, 15.0, 1.0, -0.5, 0.2],
     (0.0, 10.0)),
    (datagen.model_spec(1, 0, 2, 0.5, 2.0), [50.0, 10.0, -8.0], (-2.0, 2.0)),
    (datagen.model_spec(2, 2, -1, 0.0, 1.0),
     [300.0, 0.3, 0.04, 200.0, 0.7, 0.06, math.log(50.0), 1.0], (0.0, 1.0)),
]


def orc_model(orc, spec):
    return orc.Model(spec["kind"], spec["n_gauss"], spec["poly_degree"], spec["t_shift"],
                     spec["t_scale"])


def gpu_fisher(hf, spec, counts, theta, r, obj, weights=None):
    import torch
    yr = (r[2], r[3]) if len(r) == 4 else (0.0, 1.0)
    h = hf.make_hist(counts, (r[0], r[1]), yr, weights=weights)
    st = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    F = hf.nll_fisher(h, hf.Model.from_spec(spec), theta, objective=obj, status=st)
    torch.cuda.synchronize()
    return F.cpu().numpy(), int(st.item())


def assert_fisher(F, ref, what=""):
    d = np.sqrt(np.outer(np.abs(np.diag(ref)), np.abs(np.diag(ref))))
    err = np.abs(F - ref)
    assert np.all(err <= TOL * d), (what, float(np.max(err / np.maximum(d, 1e-300))))
    assert np.array_equal(F, F.T), what


@pytest.mark.parametrize("obj", [0, 1, 2])
@pytest.mark.parametrize("case", range(len(CASES_1D)))
def test_fisher_1d_parity(hf, orc, case, obj):
    """One bin, a tail-only 3 bins, per-bin exps (65 bins: the 16-bin chunk is
    too wide for the recurrence), and the recurrence over several blocks with
    a ragged tail; weighted and unweighted."""
    spec, th, r = CASES_1D[case]
    for nbins, weighted in ((1, False), (3, True), (65, False), (4099, True), (262147, False)):
        c = datagen.random_1d_case(spec, nbins, r[0], r[1], th, seed=2000 + nbins + case)
        counts = c["counts"]
        if nbins > 10:
            counts[::13] = 0
        w = (np.random.default_rng(nbins).uniform(0.5, 1.5, nbins).astype(np.float32)
             if weighted else None)
        ref = orc.fisher(orc_model(orc, spec), obj, counts, c["theta_eval"], r,
                         weights=None if w is None else w.astype(np.float64))
        F, st = gpu_fisher(hf, spec, counts, c["theta_eval"], r, obj, weights=w)
        assert st == 0
        assert_fisher(F, ref, (nbins, weighted))


@pytest.mark.parametrize("dtype", [np.uint32, np.float32, np.float64])
def test_fisher_neyman_count_dtypes(hf, orc, dtype):
    """Only the Neyman weight 2/n reads the counts."""
    spec, th, r = CASES_1D[0]
    c = datagen.random_1d_case(spec, 5003, r[0], r[1], th, seed=77)
    counts = c["counts"].astype(dtype)
    counts[::7] = 0
    ref = orc.fisher(orc_model(orc, spec), 0, counts.astype(np.float64), c["theta_eval"], r)
    F, st = gpu_fisher(hf, spec, counts, c["theta_eval"], r, 0)
    assert_fisher(F, ref, dtype)


def test_fisher_2d_parity(hf, orc):
    r = (0.0, 1.0, 0.0, 1.0)
    rng = np.random.default_rng(5)
    th0 = np.array([400.0, 0.45, 0.55, 0.12, 0.09, 0.3, 10.0])
    for nx, ny in ((1, 1), (37, 29), (64, 64), (513, 257), (1028, 96)):
        lam = datagen.intensity_2d(th0, nx, ny, (0, 1), (0, 1))
        counts = rng.poisson(lam).astype(np.uint32)
        w = rng.uniform(0.5, 1.5, (ny, nx)).astype(np.float32)
        th = datagen.perturb(th0, 0.02, rng)
        for obj in (0, 1, 2):
            ref = orc.fisher(orc.Model(3), obj, counts, th, r, weights=w.astype(np.float64))
            F, st = gpu_fisher(hf, datagen.model_spec(3), counts, th, r, obj, weights=w)
            assert st == 0
            assert_fisher(F, ref, (nx, ny, obj))


def test_fisher_nonfinite_theta_and_skipped_bins(hf, orc):
    spec, th, r = CASES_1D[0]
    c = datagen.random_1d_case(spec, 1000, r[0], r[1], th, seed=9)
    bad = np.array(th, dtype=np.float64)
    bad[1] = np.nan
    F, st = gpu_fisher(hf, spec, c["counts"], bad, r, 2)
    assert st == 2 and np.all(np.isnan(F))
    # a background that goes negative over part of the range: those bins have
    # c = 1/mu < 0 and are skipped by both sides
    neg = np.array([300.0, 4.8, 0.7, 20.0, -6.0])
    ref = orc.fisher(orc_model(orc, spec), 2, c["counts"], neg, r)
    F, st = gpu_fisher(hf, spec, c["counts"], neg, r, 2)
    assert st == 0
    assert_fisher(F, ref, "negative mu")


@pytest.mark.slow
def test_fisher_full_size_1e7_bins(hf, orc):
    """The 1e7-bin two-Gaussian + cubic workload (P = 10, one pass of 55
    entries), compared in full."""
    c = datagen.large_fit_case()
    spec = c["spec"]
    ref = orc.fisher(orc_model(orc, spec), 2, c["counts"], c["theta_eval"], c["range"])
    F, st = gpu_fisher(hf, spec, c["counts"], c["theta_eval"], c["range"], 2)
    assert st == 0
    assert_fisher(F, ref)


@pytest.mark.slow
def test_fisher_full_size_2048_squared(hf, orc):
    c = datagen.hist2d_case()
    r = c["range"]
    ref = orc.fisher(orc.Model(3), 2, c["counts"], c["theta_eval"], r,
                     weights=c["weights"].astype(np.float64))
    F, st = gpu_fisher(hf, c["spec"], c["counts"], c["theta_eval"], r, 2, weights=c["weights"])
    assert st == 0
    assert_fisher(F, ref)


def _cov_bound(F, cov_ref):
    d = np.sqrt(np.abs(np.diag(F)))
    R = F / np.outer(d, d)
    kappa = np.linalg.cond(R)
    s = np.sqrt(np.outer(np.abs(np.diag(cov_ref)), np.abs(np.diag(cov_ref))))
    return (1e-13 * kappa + 1e-14) * s


def test_covariance_parity_batch(hf, orc):
    """A batch of Fisher matrices from the oracle (every model size up to
    P = 16), inverted on the device, against the oracle's covariance."""
    import torch
    for obj in (0, 2):
        mats, refs = [], []
        for spec, th, r in CASES_1D:
            c = datagen.random_1d_case(spec, 3000, r[0], r[1], th, seed=31)
            F = orc.fisher(orc_model(orc, spec), obj, c["counts"], c["theta_eval"], r)
            mats.append(F)
            refs.append(orc.covariance(F, obj)[0])
        for F, ref in zip(mats, refs):
            cov, st = hf.fisher_covariance(torch.tensor(F, device="cuda"), objective=obj)
            torch.cuda.synchronize()
            assert int(st.item()) == 0
            err = np.abs(cov.cpu().numpy() - ref)
            assert np.all(err <= _cov_bound(F, ref)), F.shape
        # the same matrices as one batch (B = 4, P = 5: the first case's size)
        Fb = np.stack([orc.fisher(orc_model(orc, CASES_1D[0][0]), obj,
                                  datagen.random_1d_case(CASES_1D[0][0], 500 + 100 * b, 0.0, 10.0,
                                                         CASES_1D[0][1], seed=b)["counts"],
                                  CASES_1D[0][1], (0.0, 10.0)) for b in range(4)])
        cov, st = hf.fisher_covariance(torch.tensor(Fb, device="cuda"), objective=obj)
        torch.cuda.synchronize()
        assert st.cpu().tolist() == [0, 0, 0, 0]
        for b in range(4):
            ref = orc.covariance(Fb[b], obj)[0]
            assert np.all(np.abs(cov[b].cpu().numpy() - ref) <= _cov_bound(Fb[b], ref))


def test_covariance_free_mask_and_not_positive_definite(hf, orc):
    import torch
    F = np.array([[4.0, 1.0, 0.5], [1.0, 3.0, 0.2], [0.5, 0.2, 2.0]])
    cov, st = hf.fisher_covariance(torch.tensor(F, device="cuda"), objective=2, free_mask=0b101)
    torch.cuda.synchronize()
    ref, ok = orc.covariance(F, 2, free_mask=0b101)
    got = cov.cpu().numpy()
    assert int(st.item()) == 0 and ok
    assert np.all(got[1, :] == 0) and np.all(got[:, 1] == 0)
    assert np.all(np.abs(got - ref) <= _cov_bound(F, ref) + 0.0)
    bad = np.array([[0.999, 1.0], [1.0, 0.999]])
    cov, st = hf.fisher_covariance(torch.tensor(bad, device="cuda"), objective=0)
    torch.cuda.synchronize()
    assert int(st.item()) == 1 and np.all(np.isnan(cov.cpu().numpy()))
    assert not orc.covariance(bad, 0)[1]
    zero_diag = np.array([[1.0, 0.0], [0.0, 0.0]])
    cov, st = hf.fisher_covariance(torch.tensor(zero_diag, device="cuda"), objective=2)
    torch.cuda.synchronize()
    assert int(st.item()) == 1 and np.all(np.isnan(cov.cpu().numpy()))


def test_errors_of_a_device_fit(hf, orc):
    """Errors of fitted parameters: fit_batch on the device, then the Fisher
    matrix at each fitted theta and its covariance, against the oracle's
    Fisher matrix and covariance at the same fitted theta."""
    import torch
    spec, th, r = CASES_1D[0]
    B, nb = 6, 2000
    cases = [datagen.random_1d_case(spec, nb, r[0], r[1], th, seed=40 + b) for b in range(B)]
    counts = np.concatenate([c["counts"] for c in cases]).astype(np.uint32)
    off = np.arange(B + 1, dtype=np.int64) * nb
    ranges = np.tile(np.array(r), (B, 1))
    dev = "cuda"
    res = hf.fit_batch(torch.from_numpy(counts.view(np.int32)).to(dev),
                       torch.from_numpy(off).to(dev), torch.from_numpy(ranges).to(dev),
                       hf.Model.from_spec(spec), torch.tensor(np.tile(th, (B, 1)), device=dev))
    torch.cuda.synchronize()
    assert res.status.cpu().tolist() == [0] * B
    thetas = res.theta.cpu().numpy()
    for b in range(B):
        F, st = gpu_fisher(hf, spec, cases[b]["counts"], thetas[b], r, 2)
        ref = orc.fisher(orc_model(orc, spec), 2, cases[b]["counts"], thetas[b], r)
        assert_fisher(F, ref, b)
        cov, cst = hf.fisher_covariance(torch.tensor(F, device=dev), objective=2)
        torch.cuda.synchronize()
        cref = orc.covariance(ref, 2)[0]
        assert int(cst.item()) == 0
        assert np.all(np.abs(cov.cpu().numpy() - cref) <= _cov_bound(ref, cref) + 1e-9 * np.sqrt(
            np.outer(np.diag(cref), np.diag(cref))))

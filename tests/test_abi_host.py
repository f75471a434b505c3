"""Host-only checks of the C ABI: the library loads, exports every function
include/histfit.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "histfit.h")
LIB = os.path.join(ROOT, "paper_2203_06139_amd", "libhistfit.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhistfit.so not built; run __graft_entry__.build()")
    import paper_2203_06139_amd as hf
    return hf.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("nll_eval", "nll_grad", "fit_batch", "hf_ctx_create", "hf_ctx_destroy",
              "hf_last_error", "hf_model_nparams"):
        assert n in names, names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(ln.split()[-1] for ln in out.splitlines() if " T " in ln)
    for n in declared_functions():
        assert n in exported, n
        assert getattr(lib, n) is not None


def test_header_compiles_as_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "histfit.h"\nint main(void){hf_model m={1,1,1,0,0.0,1.0};'
                   'return hf_model_nparams(&m) == 5 ? 0 : 1;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-c", "-I", os.path.dirname(HEADER),
                    str(src), "-o", str(tmp_path / "t.o")], check=True)


def test_model_nparams(lib):
    import paper_2203_06139_amd as hf
    assert hf.Model(hf.GAUSS_POLY, 1, 1).nparams == 5
    assert hf.Model(hf.GAUSS_POLY, 2, 3, 50, 50).nparams == 10
    assert hf.Model(hf.GAUSS_EXP, 1).nparams == 5
    assert hf.Model(hf.GAUSS2D).nparams == 7
    assert hf.Model(hf.GAUSS_POLY, 4, 3).nparams == 16
    for bad in (hf.Model(hf.GAUSS_POLY, 5, 1), hf.Model(hf.GAUSS_POLY, 1, 4),
                hf.Model(hf.GAUSS_POLY, 0, -1), hf.Model(7)):
        with pytest.raises(ValueError):
            bad.nparams
    m = hf.HfModel(1, 1, 1, 0, 0.0, 0.0)  # t_scale = 0
    assert lib.hf_model_nparams(ctypes.byref(m)) == -1


def test_null_arguments_rejected_without_gpu(lib):
    assert lib.nll_eval(None, None, None, 0, 0, None, None, None, None) == -1
    assert lib.nll_grad(None, None, None, 0, 0, None, None, None, None, None, 0, None, None) == -1
    assert lib.fit_batch(None, 1, None, 0, None, None, None, 0, 0, None, None, None, None, None,
                         None, None, None) == -1
    assert lib.hf_last_error(None) == b""
    assert lib.hf_ctx_create(None, 0) == -1


def test_newer_entry_points_reject_null_context_without_gpu(lib):
    assert lib.hf_nll_fisher(None, None, None, 2, None, None, None, None) == -1
    assert lib.hf_fisher_covariance(None, 1, 5, 2, None, 0, None, None, None) == -1
    assert lib.hf_gauss_grad_map(None, 4, None, None, 0, None, 0, 0, None, None, None, None, None,
                                 None) == -1
    assert lib.nll_unbinned(None, None, None, 4, 0.0, 1.0, None, None, None, None, None,
                            None) == -1
    assert lib.hf_fit_set_wave_bins(None, 256) == -1
    assert lib.hf_fit_get_wave_bins(None) == -1
    assert lib.hf_fit_max_wave_bins(None, None, 2, 256) == -1


def test_bin_average_flag_is_validated_on_the_host(lib):
    import paper_2203_06139_amd as hf
    assert hf.Model(hf.GAUSS_POLY, 2, 3, 50, 50, bin_average=1).nparams == 10
    m = hf.HfModel(hf.GAUSS_EXP, 1, -1, 1, 0.0, 1.0)  # bin average of the exponential model
    assert lib.hf_model_nparams(ctypes.byref(m)) == 5
    m = hf.HfModel(hf.GAUSS2D, 0, -1, 1, 0.0, 1.0)  # no bin average in 2D
    assert lib.hf_model_nparams(ctypes.byref(m)) == -2
    m = hf.HfModel(hf.GAUSS_POLY, 1, 1, 2, 0.0, 1.0)  # flag must be 0 or 1
    assert lib.hf_model_nparams(ctypes.byref(m)) == -1


def test_mlp_workspace_layout_fits_the_workspace(lib):
    """The stored values' views lie inside the workspace, in carve order,
    without overlap."""
    import paper_2203_06139_amd as hf
    offs = (ctypes.c_int64 * 12)()
    assert lib.hf_mlp_workspace_layout(63, offs) == -1
    assert lib.hf_mlp_workspace_layout(64, None) == -1
    for B in (64, 192, 1024):
        assert lib.hf_mlp_workspace_layout(B, offs) == 0
        total = lib.hf_mlp_workspace_bytes(B)
        ins = (hf.MLP_IN, hf.MLP_HIDDEN, hf.MLP_HIDDEN, hf.MLP_HIDDEN)
        outs = (hf.MLP_HIDDEN, hf.MLP_HIDDEN, hf.MLP_HIDDEN, hf.MLP_OUT_PAD)
        sizes = [B * ins[l] * 2 for l in range(4)] + [B * 512 * 4] * 3 + [B * 32 * 4] + \
                [B * outs[l] * 2 for l in range(4)]
        spans = sorted(zip(list(offs), sizes))
        for (o, n), (o2, _) in zip(spans, spans[1:]):
            assert o + n <= o2
        assert all(o % 256 == 0 for o in offs)
        assert spans[-1][0] + spans[-1][1] <= total


def test_binding_rejects_host_tensors_before_any_launch():
    """Counts that are not device tensors are refused by the binding before it
    looks for a GPU, so a host pointer never reaches a kernel."""
    import numpy as np
    import torch
    import paper_2203_06139_amd as hf
    m = hf.Model(hf.GAUSS_POLY, 1, 1)
    h = hf.Hist(torch.ones(64, dtype=torch.int32), (0.0, 1.0))
    th = np.array([10.0, 0.5, 0.1, 1.0, 0.0])
    for call in (lambda: hf.nll_eval(h, m, th), lambda: hf.nll_grad(h, m, th),
                 lambda: hf.nll_fisher(h, m, th)):
        with pytest.raises(ValueError, match="device tensor"):
            call()
    with pytest.raises(ValueError, match="device tensor"):
        hf.fit_batch(torch.ones(64, dtype=torch.int32), [0, 64], [[0.0, 1.0]], m, th[None, :])

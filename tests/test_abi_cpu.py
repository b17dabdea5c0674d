"""The C-ABI library loads without a GPU, exports every symbol the public
header declares, and rejects invalid arguments on the host (no kernel is
launched for an invalid call, so these run on a CPU-only machine)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mimo_sd.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_][a-z_0-9]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_09561_amd import mimo

    if not os.path.exists(mimo.LIB_PATH):
        pytest.skip("libmimo_sd.so not built")
    return mimo.load()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("mimo_qr_preprocess", "kbest_detect", "sd_hybrid_detect", "mimo_metric", "prune_mlp_forward",
                 "prune_mlp_loss_grad", "prune_mlp_adam_step", "mimo_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2002_09561_amd import mimo

    for name in _declared():
        assert hasattr(lib, name), f"{name} declared in mimo_sd.h but not exported"
        assert name in mimo.SIGNATURES, f"{name} has no binding signature"


def _err(lib):
    return lib.mimo_last_error().decode()


def test_host_validation_without_gpu(lib):
    P = None
    # bad constellation
    assert lib.kbest_detect(P, P, 4, 4, 3, 16, P, 0, P, P, P, P, P, P) == -1
    assert "pam" in _err(lib)
    # K too large for the kernel
    assert lib.kbest_detect(P, P, 4, 4, 8, 200, P, 0, P, P, P, P, P, P) == -2
    # bad schedule stride
    assert lib.kbest_detect(P, P, 4, 4, 4, 16, ctypes.c_void_p(1), 5, P, P, P, P, P, P) == -1
    # B == 0 is a no-op even with null pointers
    assert lib.kbest_detect(P, P, 0, 4, 4, 16, P, 0, P, P, P, P, P, P) == 0
    # null pointers with B > 0
    assert lib.kbest_detect(P, P, 3, 4, 4, 16, P, 0, P, P, P, P, P, P) == -1
    # QR shape limits
    assert lib.mimo_qr_preprocess(P, P, 1, 4, 8, P, P, P, P) == -1
    assert lib.mimo_qr_preprocess(P, P, 1, 200, 100, P, P, P, P) == -2
    # hybrid limits
    assert lib.sd_hybrid_detect(P, P, 1, 4, 8, P, 16, 1, P, 0, 0, 0, P, P, P, P, P) == -1
    assert lib.sd_hybrid_detect(P, P, 1, 4, 8, P, 2, 9, P, 0, 0, 0, P, P, P, P, P) == -1
    assert lib.sd_hybrid_detect(P, P, 1, 4, 8, P, 0, 1, P, 0, 1, 0, P, P, P, P, P) == -1
    assert lib.sd_hybrid_detect(P, P, 1, 4, 8, P, 2, 2, P, 0, 0, -5, P, P, P, P, P) == -1
    # MMSE preprocessing and the linear baselines
    assert lib.mimo_qr_preprocess_mmse(P, P, P, 2, 4, 4, P, P, P) == -1
    assert "sigma2" in _err(lib)
    assert lib.mimo_qr_preprocess_mmse(P, P, P, 0, 4, 4, P, P, P) == 0
    assert lib.linear_detect(P, P, 2, 4, 3, P, P, P) == -1
    assert lib.linear_detect(P, P, 2, 200, 4, P, P, P) == -2
    assert lib.linear_detect(P, P, 2, 4, 4, P, P, P) == -1
    assert lib.mrc_detect(P, P, 2, 300, 200, 4, P, P, P) == -2
    assert lib.mrc_detect(P, P, 2, 8, 4, 4, P, P, P) == -1
    # fallback marking and selective metric
    assert lib.kbest_fallback_mark(P, P, P, 2, 4, ctypes.c_float(-1.0), P) == -1
    assert lib.kbest_fallback_mark(P, P, P, 2, 4, ctypes.c_float(3.0), P) == -1
    assert lib.mimo_metric_select(P, P, P, P, 16, 0, 2, 4, 4, 4, P, P) == -1
    assert "flags" in _err(lib)
    # MLP
    assert lib.prune_mlp_schedule(P, P, 10, 0.0, 0, 4, 8, P, P, P) == -1
    assert lib.prune_mlp_loss_grad(P, P, P, 10, 1.5, P, P, P, 0, P) == -1
    assert lib.prune_mlp_workspace_bytes(1000) >= 4 * 4 * 128 * 1000
    assert lib.mimo_version() >= 1


def test_kbest_lds_limit_and_uneven_limits(lib):
    """More than 64 survivors of 4- or 16-QAM keep their lists in LDS: K = 256
    fits the 160 KB of a compute unit up to n_tx = 77 and is refused
    (UNSUPPORTED) from n_tx = 78 on, before any launch; 64-QAM with K = 128
    fits at every size.  Uneven-batch descriptors beyond the persistent
    launch's limits are refused on the host."""
    import numpy as np

    from paper_2002_09561_amd import uneven

    P = None
    for pam in (2, 4):
        assert lib.kbest_detect(P, P, 1, 78, pam, 256, P, 0, P, P, P, P, P, P) == -2
        assert "LDS" in _err(lib)
        assert lib.kbest_detect(P, P, 1, 77, pam, 256, P, 0, P, P, P, P, P, P) == -1  # passes: null pointers
        assert lib.kbest_fallback(P, P, 1, 100, pam, 256, P, ctypes.c_float(3.0), P, P, P, P, P) == -2
        assert lib.kbest_rank_labels(P, P, 1, 90, pam, 256, P, P, P) == -2
    assert lib.kbest_detect(P, P, 1, 128, 8, 128, P, 0, P, P, P, P, P, P) == -1
    d = np.zeros(3, uneven.DESC_DTYPE)
    d["n_rx"], d["n_tx"], d["pam"], d["K"] = 16, 16, 4, 16
    uneven.validate_descriptors(d)
    for field, value in (("K", 65), ("K", 0), ("pam", 3), ("n_tx", 65), ("n_tx", 0)):
        bad = d.copy()
        bad[field][1] = value
        if field == "n_tx" and value == 65:
            bad["n_rx"][1] = 100
        with pytest.raises(ValueError):
            uneven.validate_descriptors(bad)
    bad = d.copy()
    bad["pam"][2], bad["K"][2] = 8, 64  # 512 candidates per level
    with pytest.raises(ValueError):
        uneven.validate_descriptors(bad)


def test_paper_radius_and_uneven_host_checks(lib):
    P = None
    assert lib.mimo_paper_radius2(P, 2, 4, 8, P, P) == -1   # n_rx < n_tx
    assert lib.mimo_paper_radius2(P, -1, 8, 4, P, P) == -1
    assert lib.mimo_paper_radius2(P, 0, 8, 4, P, P) == 0
    assert lib.mimo_paper_radius2(P, 3, 8, 4, P, P) == -1   # null pointers
    assert lib.kbest_detect_uneven(P, 3, P, P, P, P, P, P, 0, P) == -1
    assert lib.kbest_detect_uneven(P, 0, P, P, P, P, P, P, 0, P) == 0


def test_grouped_kbest_host_checks(lib):
    P = None
    g = lib.kbest_detect_grouped
    assert g(P, P, 1, 8, 4, 16, 3, P, 0, P, P, P, P, P, P) == -1        # J not 1 or 2
    assert "J" in _err(lib)
    assert g(P, P, 1, 8, 4, 65, 1, P, 0, P, P, P, P, P, P) == -2        # K > 64
    assert g(P, P, 1, 8, 8, 33, 2, P, 0, P, P, P, P, P, P) == -2        # 33 * 64 candidates > 2048
    assert lib.kbest_detect_complex(P, P, 1, 8, 8, 33, P, 0, P, P, P, P, P, P) == -2  # the same limit
    assert g(P, P, 1, 129, 4, 16, 1, P, 0, P, P, P, P, P, P) == -2      # n_tx > 128
    assert g(P, P, 1, 8, 3, 16, 1, P, 0, P, P, P, P, P, P) == -1        # pam
    assert g(P, P, 1, 8, 4, 16, 2, ctypes.c_void_p(1), 5, P, P, P, P, P, P) == -1  # schedule stride
    assert g(P, P, 0, 8, 4, 16, 2, P, 0, P, P, P, P, P, P) == 0          # empty batch
    assert g(P, P, 2, 8, 8, 16, 2, P, 0, P, P, P, P, P, P) == -1        # null pointers


def test_complex_hybrid_host_checks(lib):
    P = None
    g = lib.sd_hybrid_detect_complex
    assert g(P, P, 1, 4, 8, P, 2, 9, P, 0, 0, 0, P, P, P, P, P) == -1      # 9 * 64 candidates > 512
    assert "pam^2" in _err(lib)
    assert g(P, P, 1, 4, 2, P, 2, 65, P, 0, 0, 0, P, P, P, P, P) == -1     # k_worker > 64
    assert g(P, P, 1, 4, 4, P, 16, 1, P, 0, 0, 0, P, P, P, P, P) == -1     # n_workers > 15
    assert g(P, P, 1, 4, 4, P, 0, 1, P, 0, 1, 0, P, P, P, P, P) == -1      # master_off without a worker
    assert g(P, P, 1, 4, 4, P, 1, 1, ctypes.c_void_p(1), 3, 0, 0, P, P, P, P, P) == -1  # schedule stride
    assert g(P, P, 0, 4, 8, P, 2, 8, P, 0, 0, 0, P, P, P, P, P) == 0       # empty batch (8 * 64 allowed)
    assert g(P, P, 2, 4, 8, P, 2, 4, P, 0, 0, 0, P, P, P, P, P) == -1      # null pointers


def test_parallel_sd_host_checks(lib):
    P = None
    g = lib.sd_parallel_detect
    assert g(P, P, -1, 8, 4, P, 0, 0, P, P, P, P, P) == -1
    assert g(P, P, 2, 8, 5, P, 0, 0, P, P, P, P, P) == -1        # pam
    assert g(P, P, 2, 129, 4, P, 0, 0, P, P, P, P, P) == -2      # n_tx > 128
    assert g(P, P, 2, 8, 4, P, -1, 0, P, P, P, P, P) == -1       # budget < 0
    assert "budget" in _err(lib)
    assert g(P, P, 2, 8, 4, P, 0, 2, P, P, P, P, P) == -1        # redo not 0 or 1
    assert g(P, P, 0, 8, 4, P, 0, 0, P, P, P, P, P) == 0         # empty batch
    assert g(P, P, 2, 8, 4, P, 0, 0, P, P, P, P, P) == -1        # null pointers


def test_binding_refuses_cpu_tensors(lib):
    import torch

    from paper_2002_09561_amd import mimo

    with pytest.raises(TypeError):
        mimo.kbest_detect(torch.zeros(2, 36), torch.zeros(2, 8), 4, 4, 16)

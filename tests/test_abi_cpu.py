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


def test_binding_refuses_cpu_tensors(lib):
    import torch

    from paper_2002_09561_amd import mimo

    with pytest.raises(TypeError):
        mimo.kbest_detect(torch.zeros(2, 36), torch.zeros(2, 8), 4, 4, 16)

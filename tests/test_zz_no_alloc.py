"""The allocation-free loss/gradient entry point (static scratch) against the
workspace entry point it varies, through the C ABI."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(seed, S):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.3, 17281).astype(np.float32)
    X = rng.normal(size=(S, 4)).astype(np.float32)
    y = (rng.normal(size=S) * 2).astype(np.float32)
    return w, X, y


def test_noalloc_loss_grad_matches_workspace_entry_point(gpu):
    """Two calls in a row, the second with fewer states (so stale scratch of
    the first is left beyond the second's range): each equals, bit for bit,
    prune_mlp_loss_grad with a caller workspace on the same inputs; the call
    allocates no device memory; sizes beyond the scratch are refused."""
    import torch

    grad = torch.empty(17281, device="cuda")
    loss = torch.empty(1, device="cuda")
    for seed, S in ((31, 7000), (32, 1234)):
        w, X, y = (torch.from_numpy(a).cuda() for a in _case(seed, S))
        l_ref, g_ref = gpu.mlp_loss_grad(w, X, y, 0.95)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        gpu.mlp_loss_grad_noalloc(w, X, y, 0.95, grad, loss)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(grad, g_ref), S
        assert torch.equal(loss, l_ref), S
    w, X, y = (torch.from_numpy(a).cuda() for a in _case(33, gpu.MLP_NOALLOC_MAX_S + 1))
    with pytest.raises(gpu.MimoError) as ei:
        gpu.mlp_loss_grad_noalloc(w, X, y, 0.95, grad, loss)
    assert ei.value.code == gpu.ERR_UNSUPPORTED

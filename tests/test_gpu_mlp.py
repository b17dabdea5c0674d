"""GPU parity of the learned survivor-count MLP kernels against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, 17281)


def test_mlp_forward_parity(gpu, orc):
    import torch

    w = _params(1)
    X = np.random.default_rng(2).normal(size=(1000, 4))
    ref = orc.mlp_forward(w, X)
    out = gpu.mlp_forward(torch.tensor(w, dtype=torch.float32).cuda(),
                          torch.tensor(X, dtype=torch.float32).cuda()).cpu().numpy()
    # FP32 inputs and weights, FP32 accumulation over 128 terms
    wr = w.astype(np.float32).astype(np.float64)
    Xr = X.astype(np.float32).astype(np.float64)
    ref32 = orc.mlp_forward(wr, Xr)
    scale = np.maximum(1.0, np.abs(ref32))
    assert np.max(np.abs(out - ref32) / scale) < 1e-4
    assert np.max(np.abs(out - ref) / scale) < 1e-3


def test_mlp_loss_grad_parity(gpu, orc):
    import torch

    w = _params(3).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(4)
    S = 777
    X = rng.normal(size=(S, 4)).astype(np.float32).astype(np.float64)
    y = (rng.normal(size=S) * 2).astype(np.float32).astype(np.float64)
    loss_o, g_o = orc.mlp_loss_grad(w, X, y, 0.95)
    loss_g, g_g = gpu.mlp_loss_grad(torch.tensor(w, dtype=torch.float32).cuda(),
                                    torch.tensor(X, dtype=torch.float32).cuda(),
                                    torch.tensor(y, dtype=torch.float32).cuda(), 0.95)
    g_g = g_g.cpu().numpy()
    assert abs(loss_g.item() - loss_o) < 1e-4 * max(1.0, abs(loss_o))
    # per-parameter check scaled by the gradient's own magnitude
    err = np.abs(g_g - g_o)
    assert np.max(err) < 1e-4 * np.max(np.abs(g_o)) + 1e-7, np.max(err)
    # deterministic: a second call gives the identical bits
    _, g2 = gpu.mlp_loss_grad(torch.tensor(w, dtype=torch.float32).cuda(),
                              torch.tensor(X, dtype=torch.float32).cuda(),
                              torch.tensor(y, dtype=torch.float32).cuda(), 0.95)
    assert np.array_equal(g2.cpu().numpy(), g_g)


def test_adam_step_parity(gpu, orc):
    import torch

    rng = np.random.default_rng(5)
    n = 17281
    w = rng.normal(size=n).astype(np.float32).astype(np.float64)
    m = np.zeros(n)
    v = np.zeros(n)
    wt = torch.tensor(w, dtype=torch.float32).cuda()
    mt = torch.zeros(n, device="cuda")
    vt = torch.zeros(n, device="cuda")
    for t in range(1, 4):
        g = rng.normal(size=n).astype(np.float32).astype(np.float64)
        orc.adam_step(w, m, v, g, t, 1e-3)
        gpu.mlp_adam_step(wt, mt, vt, torch.tensor(g, dtype=torch.float32).cuda(), t, 1e-3)
    assert np.max(np.abs(wt.cpu().numpy() - w)) < 1e-5


def test_mlp_schedule_mapping(gpu, orc):
    import torch

    w = _params(6, 0.1)
    X = np.random.default_rng(7).normal(size=(640, 4))
    wt = torch.tensor(w, dtype=torch.float32).cuda()
    Xt = torch.tensor(X, dtype=torch.float32).cuda()
    yhat = gpu.mlp_forward(wt, Xt).cpu().numpy().astype(np.float64)
    ks = gpu.mlp_schedule(wt, Xt, n=64, margin=0.5, k_min=2, k_max=40).cpu().numpy()
    expect = np.clip(np.ceil(np.exp2(yhat + 0.5)), 2, 40)
    # exp2 in FP32 may round a value that sits on an integer either way
    assert np.all(np.abs(ks - expect) <= 1)
    assert (ks == expect).mean() > 0.99

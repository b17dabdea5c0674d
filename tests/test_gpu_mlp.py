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
    # the library's inference precision: FP32 inputs and weights, layer 2 on
    # binary16 operands (ReLU(h1), W2) with FP32 accumulation.  The oracle's
    # binary16 mode rounds the same operands (from FP64 layer-1 values); what
    # is left is FP32 accumulation over 128 terms and, rarely, an h1 that
    # FP32 and FP64 round to neighbouring halves
    wr = w.astype(np.float32).astype(np.float64)
    Xr = X.astype(np.float32).astype(np.float64)
    ref16 = orc.mlp_forward_f16(wr, Xr)
    scale = np.maximum(1.0, np.abs(ref16))
    assert np.max(np.abs(out - ref16) / scale) < 2e-4
    # against the FP64 definition: binary16 rounding of 128-term sums
    # (relative 2^-11 per operand) bounds the difference
    assert np.max(np.abs(out - ref) / np.maximum(1.0, np.abs(ref))) < 3e-2
    # tails of the batch (S not a multiple of 16) are handled
    out7 = gpu.mlp_forward(torch.tensor(w, dtype=torch.float32).cuda(),
                           torch.tensor(X[:7], dtype=torch.float32).cuda()).cpu().numpy()
    assert np.array_equal(out7, out[:7])


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
    # the same decisions taken from the oracle's forward pass in the
    # library's precision: equal except where yhat + margin lies within the
    # FP32 accumulation error of log2 of an integer
    ref16 = orc.mlp_forward_f16(w.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64))
    e = ref16 + 0.5
    expect16 = np.clip(np.ceil(np.exp2(e)), 2, 40)
    near = np.abs(np.exp2(e) - np.round(np.exp2(e))) < 2e-4 * np.exp2(e)
    assert np.all((ks == expect16) | near)

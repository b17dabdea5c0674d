"""GPU parity of the learned survivor-count MLP kernels against the FP64 oracle."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, 17281)


def _split(w):
    H = 128
    o = 0
    W1 = w[o:o + H * 4].reshape(H, 4); o += H * 4
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    w3 = w[o:o + H]; o += H
    return W1, b1, W2, b2, w3, w[o]


def mlp_error_bound(w, X):
    """Per-state bound on |f_kernel(x) - f(x)|, derived from the library's
    inference arithmetic (not fitted).  Layer 1: FP32 matrix products of 4
    terms plus the bias (gamma_6, gamma_k = k 2^-24).  Layer 2: ReLU(h1) and
    W2 are each split into two binary16 parts whose sum represents the value
    to 2^-22 relative (2^-25 absolute below the normal range), and of the
    four cross products the lo x lo one (below 2^-22 |W2| h1) is dropped: at
    most 3 2^-22 |W2| h1 + 2^-25 (|W2| + h1) per term; the 3 x 128 exact
    products and the bias are summed in FP32 (gamma_390).  Layer 3 in FP32
    (gamma_132).  ReLU is 1-Lipschitz; the factor 1.25 covers second-order
    terms.  w and X are the FP32 values the kernel reads, in FP64."""
    u32, tiny = 2.0 ** -24, 2.0 ** -25
    W1, b1, W2, b2, w3, b3 = _split(w)
    h1 = np.maximum(X @ W1.T + b1, 0)
    e1 = 6 * u32 * (np.abs(X) @ np.abs(W1).T + np.abs(b1))           # [S, H] layer-1 error
    aW2 = np.abs(W2)
    s2 = h1 @ aW2.T                                                  # sum_j |W2_ij| h1_j
    d2 = (3 * 2.0 ** -22 * s2 + tiny * (aW2.sum(1) + h1.sum(1, keepdims=True)) + e1 @ aW2.T
          + 390 * u32 * (1.002 * s2 + np.abs(b2)))
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    return 1.25 * (d2 @ np.abs(w3) + 132 * u32 * (h2 @ np.abs(w3) + abs(b3)))


def test_mlp_forward_parity(gpu, orc):
    """The kernel's output against the FP64 definition of the network on the
    same FP32 weights and inputs, state by state within the derived bound of
    the kernel's arithmetic (split-binary16 layer 2, FP32 accumulation), and
    within 1e-4 of the output's scale."""
    import torch

    w = _params(1).astype(np.float32).astype(np.float64)
    X = np.random.default_rng(2).normal(size=(1000, 4)).astype(np.float32).astype(np.float64)
    ref = orc.mlp_forward(w, X)
    out = gpu.mlp_forward(torch.tensor(w, dtype=torch.float32).cuda(),
                          torch.tensor(X, dtype=torch.float32).cuda()).cpu().numpy()
    bound = mlp_error_bound(w, X)
    err = np.abs(out - ref)
    print(f"MLP forward: max |err| / bound = {np.max(err / bound):.3f}, max rel err "
          f"{np.max(err / np.maximum(1.0, np.abs(ref))):.2e}")
    assert np.all(err <= bound)
    assert np.all(err <= 1e-4 * np.maximum(1.0, np.abs(ref)))
    # tails of the batch (S not a multiple of 16) are handled
    out7 = gpu.mlp_forward(torch.tensor(w, dtype=torch.float32).cuda(),
                           torch.tensor(X[:7], dtype=torch.float32).cuda()).cpu().numpy()
    assert np.array_equal(out7, out[:7])


@pytest.mark.parametrize("S", [777, 20000])
def test_mlp_loss_grad_parity(gpu, orc, S):
    """Loss and gradient against the FP64 oracle: 777 states (4 chunks of the
    gradient products, the last one ragged) and 20000 (the 64-chunk cap)."""
    import torch

    w = _params(3).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(4)
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
    """Survivor counts K_t = clamp(ceil(2^(f(x) + margin)), k_min, k_max)
    from the kernel against the same map of the FP64 definition f.  A state
    may differ only if f(x) + margin lies within the derived error bound
    (plus the FP32 rounding of the sum and of exp2) of log2 of an integer,
    where ceil changes its value; every other state must match exactly."""
    import torch

    w = _params(6, 0.2).astype(np.float32).astype(np.float64)
    X = np.random.default_rng(7).normal(size=(4000, 4)).astype(np.float32).astype(np.float64)
    margin, kmin, kmax = 2.5, 1, 40  # K_t spans 1 .. 15: many ceil boundaries are crossed
    wt = torch.tensor(w, dtype=torch.float32).cuda()
    Xt = torch.tensor(X, dtype=torch.float32).cuda()
    ks = gpu.mlp_schedule(wt, Xt, n=64, margin=margin, k_min=kmin, k_max=kmax).cpu().numpy()
    e = orc.mlp_forward(w, X) + margin
    expect = np.clip(np.ceil(np.exp2(e)), kmin, kmax)
    slack = mlp_error_bound(w, X) + 4 * 2.0 ** -24 * (np.abs(e) + 1.0) + 4 * 2.0 ** -23
    dist = np.min(np.abs(e[:, None] - np.log2(np.arange(1, kmax + 1))[None, :]), axis=1)
    near = dist <= slack
    print(f"MLP schedule: {int((ks != expect).sum())} of {len(ks)} differ, {int(near.sum())} near a boundary")
    assert np.all((ks == expect) | near)
    assert near.mean() < 0.03 and len(np.unique(expect)) >= 10

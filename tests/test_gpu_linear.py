"""GPU parity of the linear baselines (zero forcing, linear MMSE, MRC), the
MMSE preprocessing and MMSE-SIC, and of the paper's radius rule, against the
FP64 oracle on the same seeded frames."""
import math

import numpy as np
import pytest

from paper_2002_09561_amd.framegen import gen_frames
from tests.parity_util import check_kbest_run, check_ml, pack_level_order

pytestmark = pytest.mark.gpu


def _dev(f):
    import torch

    return torch.from_numpy(f.H).cuda(), torch.from_numpy(f.y).cuda()


def _sigma2(f):
    import torch

    return torch.full((len(f),), float(f.sigma2), device="cuda", dtype=torch.float32)


def _boundary_distance(u, P):
    """Distance of each real estimate to the nearest decision boundary of the
    PAM slicer (midpoints between neighbouring amplitudes), in amplitude units."""
    c = math.sqrt(3.0 / (2.0 * (P * P - 1)))
    v = u / c
    nb = 2.0 * np.floor(v * 0.5 + 0.5)
    nb = np.clip(nb, -(P - 2), P - 2) if P > 2 else np.zeros_like(v)
    return np.abs(v - nb) * c


def _check_linear(sym, xh, x_orc, u_orc, P, label, max_rel=1e-3):
    """xhat within max_rel of the FP64 estimate (relative to its norm); a
    symbol may differ only where the FP64 estimate of one of its two levels
    lies closer to a decision boundary than the FP32 deviation there."""
    du = np.abs(xh - u_orc)
    scale = np.sqrt((u_orc ** 2).mean(axis=1, keepdims=True)) + 1e-30
    rel = (du / scale).max(axis=1)
    print(f"{label}: max |du| / rms(u) = {rel.max():.2e}")
    assert np.all(rel <= max_rel), label
    s_orc = (x_orc[:, 0::2] * P + x_orc[:, 1::2]).astype(np.int32)
    mism = sym != s_orc
    if mism.any():
        d = _boundary_distance(u_orc, P)
        near = (d <= 4.0 * du + 1e-7)
        near_sym = near[:, 0::2] | near[:, 1::2]
        assert np.all(near_sym[mism]), f"{label}: {int((mism & ~near_sym).sum())} symbol mismatches away from a boundary"
        print(f"{label}: {int(mism.sum())} symbol mismatches at decision boundaries")
    assert mism.mean() <= 0.01, label


@pytest.mark.parametrize("N,M,q,B", [(16, 16, 16, 120), (20, 12, 64, 40), (100, 100, 64, 6)])
def test_qr_mmse_parity(gpu, orc, N, M, q, B):
    f = gen_frames(N, M, q, 10.0, B, seed=7100 + N)
    H, y = _dev(f)
    R, z = gpu.qr_preprocess_mmse(H, y, _sigma2(f))
    Ro, zo = orc.qr_mmse(f.H, f.y, float(np.float32(f.sigma2)))
    n = 2 * M
    u = 2.0 ** -24
    # ||[H; sigma I]||_F bounds the FP32 rounding of the factor
    an = np.sqrt((np.abs(f.H.astype(np.complex128)) ** 2).sum(axis=(1, 2)) * 2 + n * f.sigma2)
    yn = np.sqrt((np.abs(f.y.astype(np.complex128)) ** 2).sum(axis=1))
    err_R = np.sqrt(((R.cpu().numpy() - pack_level_order(Ro)) ** 2).sum(axis=1))
    err_z = np.sqrt(((z.cpu().numpy() - zo) ** 2).sum(axis=1))
    print(f"MMSE QR {N}x{M}: max ||dR||/||A|| = {np.max(err_R / an):.2e}, max ||dz||/||y|| = {np.max(err_z / yn):.2e}")
    assert np.all(err_R <= 8 * n * u * an)
    assert np.all(err_z <= 8 * n * u * (yn + an))


@pytest.mark.parametrize("N,M,q,snr,B", [(16, 16, 16, 14.0, 300), (20, 12, 64, 22.0, 100), (100, 100, 64, 26.0, 12)])
def test_zf_parity(gpu, orc, N, M, q, snr, B):
    f = gen_frames(N, M, q, snr, B, seed=7200 + N)
    P = math.isqrt(q)
    H, y = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    sym, xh = gpu.linear_detect(R, z, M, P, want_xhat=True)
    Ro, zo, _ = orc.qr(f.H, f.y)
    x_orc, u_orc = orc.linear(Ro, zo, P)
    _check_linear(sym.cpu().numpy(), xh.cpu().numpy(), x_orc, u_orc, P, f"ZF {N}x{M}")


@pytest.mark.parametrize("N,M,q,snr,B", [(16, 16, 16, 10.0, 300), (100, 100, 64, 22.0, 12)])
def test_linear_mmse_parity(gpu, orc, N, M, q, snr, B):
    f = gen_frames(N, M, q, snr, B, seed=7300 + N)
    P = math.isqrt(q)
    H, y = _dev(f)
    R, z = gpu.qr_preprocess_mmse(H, y, _sigma2(f))
    sym, xh = gpu.linear_detect(R, z, M, P, want_xhat=True)
    Ro, zo = orc.qr_mmse(f.H, f.y, float(np.float32(f.sigma2)))
    x_orc, u_orc = orc.linear(Ro, zo, P)
    _check_linear(sym.cpu().numpy(), xh.cpu().numpy(), x_orc, u_orc, P, f"MMSE {N}x{M}")


@pytest.mark.parametrize("N,M,q,snr,B", [(16, 16, 16, 10.0, 300), (64, 8, 64, 20.0, 200), (100, 100, 64, 26.0, 8)])
def test_mrc_parity(gpu, orc, N, M, q, snr, B):
    f = gen_frames(N, M, q, snr, B, seed=7400 + N)
    P = math.isqrt(q)
    H, y = _dev(f)
    sym, xh = gpu.mrc_detect(H, y, P, want_xhat=True)
    s_orc, u_orc = orc.mrc(f.H, f.y, q)
    xh = xh.cpu().numpy()
    assert np.allclose(xh, u_orc, rtol=1e-6, atol=1e-6)
    mism = sym.cpu().numpy() != s_orc
    if mism.any():  # only exact-boundary estimates may round differently
        d = _boundary_distance(u_orc, P)
        near = d <= 1e-9 * (1.0 + np.abs(u_orc))
        assert np.all((near[:, 0::2] | near[:, 1::2])[mism])


def test_mmse_sic_parity(gpu, orc):
    """K-best with K = 1 on the MMSE QR (MMSE successive cancellation)."""
    N = M = 16
    q, B = 16, 300
    f = gen_frames(N, M, q, 8.0, B, seed=7500)
    P = 4
    H, y = _dev(f)
    R, z = gpu.qr_preprocess_mmse(H, y, _sigma2(f))
    sym, pd, _ = gpu.kbest_detect(R, z, M, P, 1)
    Ro, zo = orc.qr_mmse(f.H, f.y, float(np.float32(f.sigma2)))
    out = orc.kbest(Ro, zo, P, 1)
    check_kbest_run(orc, "MMSE-SIC", P, 1, sym.cpu().numpy(), pd.cpu().numpy(), out, Ro, zo)
    # MMSE-SIC makes no more symbol errors than ZF-SIC on these frames
    Rz, zz = gpu.qr_preprocess(H, y)
    zf_sym, _, _ = gpu.kbest_detect(Rz, zz, M, P, 1)
    err_mmse = int((sym.cpu().numpy() != f.s_idx).sum())
    err_zf = int((zf_sym.cpu().numpy() != f.s_idx).sum())
    print(f"MMSE-SIC {err_mmse} vs ZF-SIC {err_zf} symbol errors")
    assert err_mmse <= err_zf


def test_paper_radius_exact_sd(gpu, orc):
    """The exact SD (hybrid kernel, no workers) with the paper's radius
    r^2 = N M sigma^2 (computed by the library) against the oracle's
    radius-limited SE-SD; then a radius a tenth as large, which empties the
    sphere of most frames: they are detected again without a radius on both
    sides."""
    N = M = 12
    q, B = 16, 150
    f = gen_frames(N, M, q, 6.0, B, seed=7600)
    P = 4
    H, y = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    s2 = _sigma2(f)
    r2 = gpu.paper_radius2(N, M, s2)
    assert np.array_equal(r2.cpu().numpy(), np.float32(N * M) * s2.cpu().numpy())
    Ro, zo, _ = orc.qr(f.H, f.y)
    for scale, label in ((1.0, "paper radius"), (0.1, "radius / 10")):
        r2s = (r2 * scale).contiguous()
        sym, pd, flags = gpu.sd_hybrid_detect(R, z, M, P, 0, 1, radius2=r2s)
        out = orc.sesd(Ro, zo, P, r2=r2s.cpu().numpy().astype(np.float64))
        fl = flags.cpu().numpy()
        assert np.all(fl & orc.FOUND) and np.all(out[2] & orc.FOUND)
        assert np.array_equal(fl & orc.EMPTY_SPHERE, out[2] & orc.EMPTY_SPHERE), label
        if scale < 1.0:
            assert np.any(fl & orc.EMPTY_SPHERE)
        check_ml(orc, label, P, sym.cpu().numpy(), out, f.H, f.y, q)

"""GPU parity: QR preprocessing, batched K-best, labels and epilogues against
the FP64 oracle on the same seeded frames."""
import math

import numpy as np
import pytest

from paper_2002_09561_amd.framegen import gen_frames
from tests.parity_util import check_kbest, check_kbest_run, pack_level_order

pytestmark = pytest.mark.gpu


def _dev(frames):
    import torch

    return (torch.from_numpy(frames.H).cuda(), torch.from_numpy(frames.y).cuda(),
            torch.from_numpy(frames.s_idx).cuda())


def _np(t):
    return t.cpu().numpy()


# ----------------------------------------------------------------- QR
@pytest.mark.parametrize("N,M,q,B", [(4, 4, 4, 37), (16, 16, 16, 130), (20, 12, 64, 9), (32, 32, 16, 64),
                                     (100, 100, 64, 6), (128, 128, 4, 3), (1, 1, 16, 5)])
def test_qr_parity(gpu, orc, N, M, q, B):
    f = gen_frames(N, M, q, 18.0, B, seed=1000 + N + M)
    H, y, _ = _dev(f)
    R, z, resid = gpu.qr_preprocess(H, y, want_resid=True)
    Ro, zo, reso = orc.qr(f.H, f.y)
    Rp = pack_level_order(Ro)
    n = 2 * M
    # the FP64 Cholesky-QR factor rounded to FP32: ||dR|| <= c n u ||H||, u = 2^-24
    # (the FP64 error, amplified by cond(H)^2, is far below the FP32 rounding)
    u = 2.0 ** -24
    hn = np.sqrt((np.abs(f.H.astype(np.complex128)) ** 2).sum(axis=(1, 2)) * 2)
    err_R = np.sqrt(((_np(R) - Rp) ** 2).sum(axis=1))
    err_z = np.sqrt(((_np(z) - zo) ** 2).sum(axis=1))
    yn = np.sqrt((np.abs(f.y.astype(np.complex128)) ** 2).sum(axis=1))
    print(f"QR {N}x{M}: max ||dR||/||H|| = {np.max(err_R / hn):.2e}, max ||dz||/||y|| = {np.max(err_z / yn):.2e}")
    assert np.all(err_R <= 8 * n * u * hn)
    assert np.all(err_z <= 8 * n * u * (yn + hn))
    assert np.all(np.abs(_np(resid) - reso) <= 8 * n * u * yn ** 2 + 1e-6)
    # exact zeros of the interleaved structure: R_{2k,2k+1} = 0
    Rg = _np(R)
    for k in range(0, n, 2):
        off = (n - 1 - k) * (n - k) // 2
        assert np.all(Rg[:, off + 1] == 0.0)


@pytest.mark.parametrize("M", [2, 3, 7, 15, 31, 47, 64, 72, 73, 96, 97, 104, 107, 111, 127])
def test_qr_parity_sizes(gpu, orc, M):
    """Sizes across the kernel's launch shapes: one frame per workgroup (up to
    3 and from 7 waves), two per workgroup (4 to 6 waves, an odd batch leaves
    the second half of the last workgroup idle), the compile-time tile-row
    counts (M = 64) and the generic ones, and the step from which the last
    wave runs the Cholesky alone; N > M on every other size."""
    N = min(128, M + (M % 2) * 3)
    B = 3
    f = gen_frames(N, M, 16, 15.0, B, seed=1500 + M)
    H, y, _ = _dev(f)
    R, z, resid = gpu.qr_preprocess(H, y, want_resid=True)
    Ro, zo, reso = orc.qr(f.H, f.y)
    n = 2 * M
    u = 2.0 ** -24
    hn = np.sqrt((np.abs(f.H.astype(np.complex128)) ** 2).sum(axis=(1, 2)) * 2)
    yn = np.sqrt((np.abs(f.y.astype(np.complex128)) ** 2).sum(axis=1))
    err_R = np.sqrt(((_np(R) - pack_level_order(Ro)) ** 2).sum(axis=1))
    err_z = np.sqrt(((_np(z) - zo) ** 2).sum(axis=1))
    assert np.all(err_R <= 8 * n * u * hn), f"{N}x{M}"
    assert np.all(err_z <= 8 * n * u * (yn + hn)), f"{N}x{M}"
    assert np.all(np.abs(_np(resid) - reso) <= 8 * n * u * yn ** 2 + 1e-6), f"{N}x{M}"


def _unpack_level_order(Rp, n):
    """Packed level order [B, n(n+1)/2] -> full upper-triangular [B, n, n]."""
    R = np.zeros((Rp.shape[0], n, n))
    off = 0
    for k in range(n - 1, -1, -1):
        R[:, k, k:] = Rp[:, off: off + n - k]
        off += n - k
    return R


def _real_embedding(H):
    """Complex [B, N, M] -> real [B, 2N, 2M] with 2x2 blocks [[a, -b], [b, a]]
    (entry j of s at real indices 2j, 2j + 1, as in the level order)."""
    B, N, M = H.shape
    Hr = np.zeros((B, 2 * N, 2 * M))
    Hr[:, 0::2, 0::2] = H.real
    Hr[:, 0::2, 1::2] = -H.imag
    Hr[:, 1::2, 0::2] = H.imag
    Hr[:, 1::2, 1::2] = H.real
    return Hr


@pytest.mark.parametrize("N,M", [(16, 16), (100, 100)])
def test_qr_rank_deficient(gpu, orc, N, M):
    """Channels with a zero column (at a tile edge, inside a tile, the last
    one) or two equal columns.  The factor is then not unique, so what is
    checked is what every valid one satisfies: R^T R = H^T H and R^T z = H^T y
    for the real model, rho^2 = ||y||^2 - ||z||^2 >= 0, all finite, and a zero
    column gives an exactly zero row and column of R.  The healthy first frame
    pins the real embedding against the oracle's factor."""
    B = 5
    f = gen_frames(N, M, 64, 20.0, B, seed=1700 + M)
    H = f.H.copy()
    zero_cols = {1: 4, 2: 6, 3: M - 1}  # frame -> zeroed column
    for b, j in zero_cols.items():
        H[b, :, j] = 0
    H[4, :, M // 2] = H[4, :, 1]
    import torch

    R, z, resid = gpu.qr_preprocess(torch.from_numpy(H).cuda(), torch.from_numpy(f.y).cuda(), want_resid=True)
    n = 2 * M
    Rf = _unpack_level_order(_np(R).astype(np.float64), n)
    zf = _np(z).astype(np.float64)
    rs = _np(resid).astype(np.float64)
    assert np.all(np.isfinite(Rf)) and np.all(np.isfinite(zf)) and np.all(np.isfinite(rs))
    Hr = _real_embedding(H.astype(np.complex128))
    yr = np.zeros((B, 2 * N))
    yr[:, 0::2] = f.y.real
    yr[:, 1::2] = f.y.imag
    u = 2.0 ** -24
    y2 = (yr ** 2).sum(axis=1)
    G = np.einsum("bki,bkj->bij", Hr, Hr)
    Gq = np.einsum("bki,bkj->bij", Rf, Rf)
    hy = np.einsum("bki,bk->bi", Hr, yr)
    rz = np.einsum("bki,bk->bi", Rf, zf)
    d = np.sqrt(np.einsum("bii->bi", G))  # column norms of the real H
    # per entry: the FP32 rounding of R and z, c n u |h_i| |h_j| (0 for a zero column)
    for b in range(B):
        assert np.all(np.abs(Gq[b] - G[b]) <= 4 * n * u * np.outer(d[b], d[b])), b
        assert np.all(np.abs(rz[b] - hy[b]) <= 4 * n * u * d[b] * np.sqrt(y2[b])), b
        assert rs[b] >= 0.0 and abs(rs[b] - (y2[b] - (zf[b] ** 2).sum())) <= 16 * n * u * y2[b], b
    for b, j in zero_cols.items():
        assert np.all(Rf[b, 2 * j: 2 * j + 2, :] == 0.0) and np.all(Rf[b, :, 2 * j: 2 * j + 2] == 0.0), b
        assert np.all(zf[b, 2 * j: 2 * j + 2] == 0.0), b
    # the healthy frame against the oracle's factor (unique there)
    Ro, zo, _ = orc.qr(f.H[:1], f.y[:1])
    assert np.max(np.abs(Rf[0] - Ro[0])) <= 8 * n * u * np.sqrt((d[0] ** 2).sum())


@pytest.mark.parametrize("N,M,q", [(1, 1, 4), (3, 3, 16), (6, 5, 64), (7, 7, 4), (13, 12, 16), (33, 33, 64),
                                   (100, 100, 64), (128, 127, 16), (40, 8, 64)])
def test_metric_parity_sizes(gpu, orc, N, M, q):
    """FP64 metric ||y - H s||^2 of random symbols: even n_tx takes the
    16-byte loads (two columns), odd n_tx the single-column path; n_rx > n_tx
    and rows not a multiple of the row groups."""
    import torch

    B = 7
    f = gen_frames(N, M, q, 12.0, B, seed=1600 + N + M)
    H, y, _ = _dev(f)
    rng = np.random.default_rng(N * 1000 + M)
    s = rng.integers(0, q, (B, M)).astype(np.int32)
    P = math.isqrt(q)
    m_gpu = _np(gpu.metric(H, y, torch.from_numpy(s).cuda(), P))
    m_orc = orc.metric(f.H, f.y, s, q)
    assert np.allclose(m_gpu, m_orc, rtol=1e-10, atol=1e-12), f"{N}x{M}"


# ----------------------------------------------------------------- K-best
def _kbest_case(gpu, orc, N, M, q, snr, B, K, seed, radius=None, sched=None):
    import torch

    f = gen_frames(N, M, q, snr, B, seed=seed)
    P = math.isqrt(q)
    n = 2 * M
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    r2 = None if radius is None else torch.from_numpy(radius.astype(np.float32)).cuda()
    ks = None if sched is None else torch.from_numpy(sched.astype(np.int32)).cuda()
    print(f"K-best {N}x{M} {q}-QAM {snr} dB B={B} K={K} radius={radius is not None} sched={sched is not None}",
          flush=True)
    sym, pd, flags, ctr = gpu.kbest_detect(R, z, M, P, K, k_sched=ks, radius2=r2, want_counters=True)
    Ro, zo, reso = orc.qr(f.H, f.y)
    if radius is None:
        out = orc.kbest(Ro, zo, P, K, k_sched=sched)
    else:  # per-frame radius (the FP32 value the GPU compares with): frame by frame
        parts = [orc.kbest(Ro[b:b + 1], zo[b:b + 1], P, K, k_sched=None if sched is None else sched[b:b + 1],
                           r2=float(np.float32(radius[b]))) for b in range(B)]
        out = {k: np.concatenate([p[k] for p in parts]) for k in ("x", "pd", "margin", "flags", "counters")}
    return f, P, n, out, (sym, pd, flags, ctr), (Ro, zo, reso)


def _forced_per_frame(orc, Ro, zo, P, K, radius, sched=None):
    """forced(mask, x) for frames with their own radius."""
    def forced(mask, xf):
        idx = np.nonzero(mask)[0]
        return np.array([orc.kbest(Ro[b:b + 1], zo[b:b + 1], P, K, r2=float(np.float32(radius[b])),
                                   k_sched=None if sched is None else sched[b:b + 1],
                                   force_path=xf[i:i + 1])["fgap"][0] for i, b in enumerate(idx)])
    return forced


@pytest.mark.parametrize("M,q,snr,B,K", [(4, 4, 10.0, 1000, 16), (16, 16, 4.0, 300, 64), (16, 16, 12.0, 300, 64),
                                         (16, 16, 20.0, 257, 64), (8, 64, 18.0, 200, 5), (10, 16, 8.0, 150, 1),
                                         (32, 16, 14.0, 100, 16), (6, 4, 6.0, 100, 256), (12, 64, 20.0, 61, 128),
                                         (1, 16, 5.0, 50, 3)])
def test_kbest_parity(gpu, orc, M, q, snr, B, K):
    f, P, n, out, (sym, pd, flags, ctr), (Ro, zo, reso) = _kbest_case(gpu, orc, M, M, q, snr, B, K,
                                                                      seed=2000 + M + K)
    eps, tol, nm = check_kbest_run(orc, f"K-best {M}x{M} {q}-QAM K={K} {snr}dB", P, K, _np(sym), _np(pd), out,
                                   Ro, zo)
    assert nm <= max(3, B // 20)
    assert np.all(_np(flags) & 1)
    # node counters follow the closed form sum_t min(K, P^t)
    expect = sum(min(K, P ** t) for t in range(n))
    assert np.all(_np(ctr)[:, 0] == expect) and np.all(_np(ctr)[:, 1] == P * expect)
    # FP64 metric epilogue of the same symbols
    H, y, _ = _dev(f)
    m_gpu = _np(gpu.metric(H, y, sym, P))
    m_orc = orc.metric(f.H, f.y, _np(sym), q)
    assert np.allclose(m_gpu, m_orc, rtol=1e-10, atol=1e-12)


def test_kbest_large_K_and_K1(gpu, orc):
    """K = 256 (a survivor list in LDS) and K = 1 (successive cancellation)
    against the oracle's K-best at the same K; the oracle's K = 1 is the SIC
    slicer (pinned on the CPU)."""
    f = gen_frames(4, 4, 16, 8.0, 200, seed=2100)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    Ro, zo, _ = orc.qr(f.H, f.y)
    for K in (256, 1):
        sym, pd, _ = gpu.kbest_detect(R, z, 4, 4, K)
        check_kbest_run(orc, f"4x4 16-QAM K={K}", 4, K, _np(sym), _np(pd), orc.kbest(Ro, zo, 4, K), Ro, zo)


def test_kbest_radius_and_empty_sphere(gpu, orc):
    """Per-frame radius around the ML metric: frames whose sphere is empty
    are detected again without a radius (EMPTY_SPHERE with FOUND) in both
    implementations; the flag agrees except where the radius test itself was
    a near tie; counters add up both searches."""
    B = 120
    f = gen_frames(8, 8, 16, 10.0, B, seed=2200)
    Ro, zo, _ = orc.qr(f.H, f.y)
    ml = orc.sesd(Ro, zo, 4)[1]
    rng = np.random.default_rng(5)
    radius = ml * rng.uniform(0.6, 2.0, size=B)  # some frames below the ML metric
    f2, P, n, out, (sym, pd, flags, ctr), _ = _kbest_case(gpu, orc, 8, 8, 16, 10.0, B, 8, seed=2200,
                                                          radius=radius)
    fl, of = _np(flags), out["flags"]
    empty_o, empty_g = (of & 2) != 0, (fl & 2) != 0
    assert np.all(fl & 1) and np.all(of & 1)
    assert empty_o.any() and (~empty_o).any()
    near = out["margin"][:, 0] <= 1e-4  # a radius test this close may fall either way in FP32
    assert np.all((empty_o == empty_g) | near)
    ok = empty_o == empty_g
    forced = _forced_per_frame(orc, Ro[ok], zo[ok], P, 8, radius[ok])
    check_kbest(orc, "radius", P, orc.sym_to_x(_np(sym)[ok], P), _np(pd)[ok],
                {k: out[k][ok] for k in ("x", "pd")}, Ro[ok], zo[ok], forced)
    # counters: a re-detected frame adds a second, unpruned search to the first
    per = sum(min(8, P ** t) for t in range(n))
    c = _np(ctr)[:, 0]
    assert np.all(c[empty_g] > per)
    clean = out["margin"][:, 0] > 1e-4
    assert np.array_equal(c[clean], out["counters"][clean, 0])


def test_kbest_per_frame_schedule(gpu, orc):
    B, M = 100, 16
    rng = np.random.default_rng(6)
    sched = rng.integers(1, 33, size=(B, 2 * M)).astype(np.int32)
    f, P, n, out, (sym, pd, flags, ctr), (Ro, zo, _) = _kbest_case(gpu, orc, M, M, 16, 10.0, B, 32, seed=2300,
                                                                   sched=sched)
    check_kbest_run(orc, "schedule", P, 32, _np(sym), _np(pd), out, Ro, zo, k_sched=sched)
    # expanded nodes follow the schedule: 1 + sum over levels of min(K_t, P * previous)
    exp = np.zeros(B, np.int64)
    for b in range(B):
        cnt = 1
        for k in range(n - 1, -1, -1):
            exp[b] += cnt
            cnt = min(sched[b, k], cnt * P)
    assert np.array_equal(_np(ctr)[:, 0], exp)


@pytest.mark.parametrize("M,snr,B,K", [(40, 16.0, 101, 8), (100, 24.0, 13, 6), (33, 14.0, 64, 3), (104, 26.0, 5, 8)])
def test_kbest_two_frames_per_wave(gpu, orc, M, snr, B, K):
    """64-QAM with at most 8 survivors and 64 < n <= 208 runs two frames per
    wavefront (the learned detector's case): parity with the oracle under a
    per-frame schedule, expanded-node counts on every frame, and an odd
    batch whose last wavefront has an idle half."""
    rng = np.random.default_rng(M + K)
    n = 2 * M
    sched = rng.integers(1, K + 1, size=(B, n)).astype(np.int32)
    f, P, n, out, (sym, pd, flags, ctr), (Ro, zo, _) = _kbest_case(gpu, orc, M, M, 64, snr, B, K, seed=2350 + M,
                                                                   sched=sched)
    check_kbest_run(orc, f"two frames per wave {M}x{M}", P, K, _np(sym), _np(pd), out, Ro, zo, k_sched=sched)
    assert np.array_equal(_np(ctr)[:, :2], out["counters"][:, :2])
    assert np.all((_np(flags) & gpu.FLAG_FOUND) != 0)


def test_kbest_two_frames_per_wave_radius(gpu, orc):
    """Per-frame radius on the two-frames-per-wave kernel: a frame whose
    sphere empties ends there while its partner goes on, and the re-run
    without a radius (one frame per wave) completes it."""
    M, B, K = 40, 61, 4
    f = gen_frames(M, M, 64, 16.0, B, seed=2400)
    Ro, zo, _ = orc.qr(f.H, f.y)
    ref = orc.kbest(Ro, zo, 8, K)
    rng = np.random.default_rng(7)
    radius = ref["pd"] * rng.uniform(0.3, 1.6, size=B)  # some spheres hold no K-best leaf
    f2, P, n, out, (sym, pd, flags, ctr), _ = _kbest_case(gpu, orc, M, M, 64, 16.0, B, K, seed=2400, radius=radius)
    fl = _np(flags)
    empty_o, empty_g = (out["flags"] & 2) != 0, (fl & 2) != 0
    near = out["margin"][:, 0] <= 1e-4
    assert np.all((empty_o == empty_g) | near)
    assert empty_o.any() and (~empty_o).any()
    assert np.all(fl & 1)
    ok = empty_o == empty_g
    forced = _forced_per_frame(orc, Ro[ok], zo[ok], P, K, radius[ok])
    check_kbest(orc, "pair radius", P, orc.sym_to_x(_np(sym)[ok], P), _np(pd)[ok],
                {k: out[k][ok] for k in ("x", "pd")}, Ro[ok], zo[ok], forced)


@pytest.mark.parametrize("K", [16, 64, 3])
def test_rank_labels_parity(gpu, orc, K):
    """Labels (1-based rank of the ML prefix at each level) are integers and
    must match exactly, except at a level whose rank, or an earlier
    selection, hinged on two keys within the near-tie window (oracle rgap,
    logged)."""
    import torch

    B, M, q = 80, 8, 16
    f = gen_frames(M, M, q, 8.0, B, seed=2400)
    P, n = 4, 16
    Ro, zo, _ = orc.qr(f.H, f.y)
    ml = orc.sesd(Ro, zo, P)[0]
    out = orc.kbest(Ro, zo, P, K, force_path=ml)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    sym, pd, _ = gpu.kbest_detect(R, z, M, P, K)
    _, tol, _ = check_kbest_run(orc, f"rank-label frames K={K}", P, K, _np(sym), _np(pd), orc.kbest(Ro, zo, P, K),
                                Ro, zo)
    rank = _np(gpu.kbest_rank_labels(R, z, M, P, K, torch.from_numpy(orc.x_to_sym(ml, P)).cuda()))
    # a level is exposed to a near tie if it or any level above it had one
    exposed = np.minimum.accumulate(out["rgap"][:, ::-1], axis=1)[:, ::-1] <= tol
    diff = rank != out["rank"]
    print(f"rank labels K={K}: {diff.sum()} of {diff.size} differ, {exposed.sum()} levels exposed to near ties")
    assert not np.any(diff & ~exposed)


# ----------------------------------------------------------------- epilogues
def test_error_count_parity(gpu, orc):
    import torch

    rng = np.random.default_rng(7)
    for q, M, B in ((4, 4, 100), (16, 16, 333), (64, 100, 40)):
        P = math.isqrt(q)
        ref = rng.integers(0, q, size=(B, M)).astype(np.int32)
        hat = ref.copy()
        flip = rng.random((B, M)) < 0.05
        hat[flip] = rng.integers(0, q, size=flip.sum())
        c = _np(gpu.error_count(torch.from_numpy(hat).cuda(), torch.from_numpy(ref).cuda(), P))
        bits, syms = orc.error_counts(hat, ref, P)
        assert c[0] == bits and c[1] == syms and c[2] == int(np.any(hat != ref, axis=1).sum())


@pytest.mark.parametrize("M,q,B", [(16, 16, 64), (7, 64, 37), (33, 4, 21), (100, 64, 30), (128, 16, 6)])
def test_prune_features_parity(gpu, orc, M, q, B):
    """Every frame, every level.  Sizes with n = 2 n_tx a multiple of 4 and
    not (the kernel's row buffers then leave two levels), both slot counts
    (13 up to 208 levels, 16 above), and batches that leave the last wave's
    four frames partly empty.  The features follow the successive-
    cancellation path; the two paths may part only at a level whose centre
    lies within its FP32 rounding bound of a decision boundary (f1 ~ 0 on
    the oracle's side), and there only levels from that one down may
    differ."""
    import torch

    P = math.isqrt(q)
    n = 2 * M
    f = gen_frames(M, M, q, 14.0, B, seed=2500 + M)
    Ro, zo, _ = orc.qr(f.H, f.y)
    fo = orc.prune_features(Ro, zo, P, f.sigma2)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    s2 = torch.full((B,), f.sigma2, device="cuda", dtype=torch.float32)
    fg = _np(gpu.prune_features(R, z, s2, M, P))
    assert fg.shape == fo.shape
    d = np.abs(fg - fo)
    ok = ((d[..., 0] < 1e-6) & (d[..., 1] < 1e-3) & (d[..., 2] < 1e-4)
          & (d[..., 3] < 1e-3 * np.maximum(1.0, np.abs(fo[..., 3]))))
    # FP32 rounding bound of each centre in units of the spacing 2c, along
    # the oracle's path: (terms + 4) u (|z_k| + sum_j |R_kj a_j|) / (R_kk 2c)
    xs, _ = orc.zf_sic(Ro, zo, P)
    c = orc.pam_scale(P)
    amp = (2.0 * xs - (P - 1)) * c
    S = np.abs(zo) + np.abs(np.triu(Ro, 1) * amp[:, None, :]).sum(axis=2)
    terms = (n - 1 - np.arange(n))[None, :]
    slice_tol = (terms + 4) * 2.0 ** -24 * S / (np.einsum("bkk->bk", Ro) * 2 * c) + 1e-7
    parted = 0
    for b in range(B):
        bad = np.nonzero(~ok[b])[0]
        if bad.size == 0:
            continue
        k0 = bad.max()  # the highest level that differs: the paths part there
        assert fo[b, k0, 1] <= slice_tol[b, k0], (b, k0, fo[b, k0], fg[b, k0])
        parted += 1
    print(f"features {M}x{M} {q}-QAM: {parted} of {B} frames part at a near tie")
    assert parted <= max(2, B // 10)


@pytest.mark.parametrize("M", [100, 128])
def test_prune_features_frames_isolated(gpu, M):
    """A wave computes the features of four frames and its lanes may read
    entries of a neighbouring frame's R (which meet a zero amplitude): a
    non-finite frame must leave every other frame's features unchanged."""
    import torch

    B = 8
    f = gen_frames(M, M, 64, 20.0, B, seed=2550 + M)
    H, y, _ = _dev(f)
    s2 = torch.full((B,), f.sigma2, device="cuda", dtype=torch.float32)
    R, z = gpu.qr_preprocess(H, y)
    clean = _np(gpu.prune_features(R, z, s2, M, 8))
    for bad in (0, 2, 3, 7):  # first, inside and last of a wave of four, last frame
        Hb = H.clone()
        Hb[bad, 1, 2] = float("nan")
        Rb, zb = gpu.qr_preprocess(Hb, y)
        fb = _np(gpu.prune_features(Rb, zb, s2, M, 8))
        for i in range(B):
            if i != bad:
                assert np.array_equal(fb[i], clean[i]), (bad, i)


# ----------------------------------------------------------------- full size, sampled
def test_kbest_100x100_64qam_sampled(gpu, orc):
    """The benchmark's shape (100x100 64-QAM, K = 16) in its launch
    configuration; a sample of frames is checked against the oracle."""
    B = 512
    f = gen_frames(100, 100, 64, 20.0, B, seed=2600)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    sym, pd, flags = gpu.kbest_detect(R, z, 100, 8, 16)
    idx = np.arange(0, B, 16)
    Ro, zo, _ = orc.qr(f.H[idx], f.y[idx])
    out = orc.kbest(Ro, zo, 8, 16)
    check_kbest_run(orc, "100x100 K=16", 8, 16, _np(sym)[idx], _np(pd)[idx], out, Ro, zo)
    m = _np(gpu.metric(H, y, sym, 8))
    mo = orc.metric(f.H[idx], f.y[idx], _np(sym)[idx], 64)
    assert np.allclose(m[idx], mo, rtol=1e-10)


def test_kbest_fallback(gpu, orc):
    """Frames whose first detection (here K = 1) is above the noise bound, or
    flagged, are detected again by plain K-best; the others are untouched."""
    import torch

    B, M, q = 200, 16, 16
    f = gen_frames(M, M, q, 10.0, B, seed=2700)
    P, n = 4, 2 * M
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    sym, pd, flags = gpu.kbest_detect(R, z, M, P, 1)
    flags[:5] |= gpu.FLAG_LEARNED_FALLBACK  # forced fallback on the first frames
    first = (_np(sym).copy(), _np(pd).copy(), _np(flags).copy())
    s2 = torch.full((B,), f.sigma2, device="cuda", dtype=torch.float32)
    beta = 3.0
    gpu.kbest_fallback(R, z, M, P, 32, s2, beta, (sym, pd, flags))
    bound = 0.5 * np.float32(f.sigma2) * (n + beta * np.sqrt(2 * n))
    redo = ((first[2] & gpu.FLAG_LEARNED_FALLBACK) != 0) | (first[1] > bound)
    assert redo.any() and (~redo).any()
    fl = _np(flags)
    assert np.all(((fl & gpu.FLAG_LEARNED_FALLBACK) != 0) == redo)
    assert np.array_equal(_np(sym)[~redo], first[0][~redo])
    assert np.array_equal(_np(pd)[~redo], first[1][~redo])
    Ro, zo, _ = orc.qr(f.H, f.y)
    kb = orc.kbest(Ro[redo], zo[redo], P, 32)
    check_kbest_run(orc, "fallback", P, 32, _np(sym)[redo], _np(pd)[redo], kb, Ro[redo], zo[redo])


@pytest.mark.parametrize("M,snr,B,K", [(16, 14.0, 200, 64), (16, 10.0, 120, 40), (40, 18.0, 60, 64),
                                       (100, 22.0, 8, 64)])
def test_kbest_fallback_64qam(gpu, orc, M, snr, B, K):
    """64-QAM fallback with 33..64 survivors (the learned detector's case):
    the re-detected frames equal the oracle's K-best (up to near ties) and
    plain K-best's result on the same frames, with the same expanded-node
    counts; the other frames keep their first detection."""
    import torch

    q, P, n = 64, 8, 2 * M
    f = gen_frames(M, M, q, snr, B, seed=2800 + M + K)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    sym, pd, flags = gpu.kbest_detect(R, z, M, P, 1)
    flags[::2] |= gpu.FLAG_LEARNED_FALLBACK  # half the frames forced
    first_flags = _np(flags).copy()
    first_sym = _np(sym).copy()
    s2 = torch.full((B,), f.sigma2, device="cuda", dtype=torch.float32)
    ctr = torch.zeros(B, 4, device="cuda", dtype=torch.int64)
    print(f"fallback {M}x{M} 64-QAM K={K} B={B}", flush=True)
    gpu.kbest_fallback(R, z, M, P, K, s2, 3.0, (sym, pd, flags), counters=ctr)
    redo = (_np(flags) & gpu.FLAG_LEARNED_FALLBACK) != 0
    assert np.all(redo[::2])
    assert np.array_equal(_np(sym)[~redo], first_sym[~redo])
    # the one-wave K-best on the same frames
    s1, p1, f1, c1 = gpu.kbest_detect(R, z, M, P, K, want_counters=True)
    Ro, zo, _ = orc.qr(f.H, f.y)
    kb = orc.kbest(Ro[redo], zo[redo], P, K)
    _, tol, _ = check_kbest_run(orc, "64-QAM fallback", P, K, _np(sym)[redo], _np(pd)[redo], kb, Ro[redo],
                                zo[redo])
    clean = kb["margin"][:, 0] > tol
    assert np.array_equal(_np(ctr)[redo][clean, :2], kb["counters"][clean, :2])
    assert np.array_equal(_np(sym)[redo][clean], _np(s1)[redo][clean])
    assert np.allclose(_np(pd)[redo][clean], _np(p1)[redo][clean], rtol=5e-5)
    assert np.all((_np(flags)[redo] & gpu.FLAG_FOUND) != 0)


def test_fallback_mark_and_metric_select(gpu):
    """kbest_fallback_mark flags exactly the frames kbest_fallback detects
    again (and changes nothing else); mimo_metric_select writes the metric of
    the selected frames only, equal to the full metric there."""
    import torch

    M, q, B, P = 16, 16, 400, 4
    f = gen_frames(M, M, q, 8.0, B, seed=2700)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    s2 = torch.full((B,), f.sigma2, device="cuda", dtype=torch.float32)
    sym, pd, flags = gpu.kbest_detect(R, z, M, P, 1)
    beta = 2.0
    fl_mark = flags.clone()
    gpu.kbest_fallback_mark(M, s2, beta, (sym, pd, fl_mark))
    s_fb, pd_fb, fl_fb = sym.clone(), pd.clone(), flags.clone()
    gpu.kbest_fallback(R, z, M, P, 16, s2, beta, (s_fb, pd_fb, fl_fb))
    FB = gpu.FLAG_LEARNED_FALLBACK
    marked = (_np(fl_mark) & FB) != 0
    assert 0 < marked.sum() < B
    assert np.array_equal(marked, (_np(fl_fb) & FB) != 0)
    assert np.array_equal(_np(fl_mark)[~marked], _np(flags)[~marked])
    assert np.array_equal(_np(s_fb)[~marked], _np(sym)[~marked])
    full = gpu.metric(H, y, s_fb, P)
    out = torch.full((B,), float("nan"), device="cuda", dtype=torch.float64)
    gpu.metric_select(H, y, s_fb, P, fl_mark, FB, 0, out)
    o = _np(out)
    assert np.array_equal(o[~marked], _np(full)[~marked]) and np.all(np.isnan(o[marked]))
    gpu.metric_select(H, y, s_fb, P, fl_mark, FB, FB, out)
    assert np.array_equal(_np(out), _np(full))


# ----------------------------------------------------------------- non-finite input
@pytest.mark.parametrize("M,q,K,variant", [(16, 16, 16, "register"), (40, 64, 4, "two frames per wave"),
                                           (8, 16, 128, "survivor lists in LDS"), (16, 64, 10, "complex levels"),
                                           (12, 16, 1, "hybrid W=0"), (12, 16, 4, "hybrid W=3")])
def test_nonfinite_input(gpu, orc, M, q, K, variant):
    """A NaN in H (which spreads through the QR) or an infinity planted in R
    at a low level: the frame ends at the first level that meets it with
    flags NONFINITE_INPUT and nothing else, sym 0 and pd +inf; every other
    frame's result, flags and counters are those of the clean batch."""
    import torch

    B = 12
    P = math.isqrt(q)
    f = gen_frames(M, M, q, 16.0, B, seed=2900 + M)
    H, y, _ = _dev(f)
    n = 2 * M
    R, z = gpu.qr_preprocess(H, y)

    def run(R, z):
        print(f"non-finite {variant} {M}x{M} {q}-QAM K={K}", flush=True)
        if variant.startswith("hybrid"):
            W = 0 if variant.endswith("0") else 3
            return gpu.sd_hybrid_detect(R, z, M, P, W, K, node_budget=200000, want_counters=True)
        if variant == "complex levels":
            return gpu.kbest_detect_complex(R, z, M, P, K, want_counters=True)
        return gpu.kbest_detect(R, z, M, P, K, want_counters=True)

    clean = [_np(t) for t in run(R, z)]
    Hb = H.clone()
    Hb[1, 3, 2] = float("nan")
    Rb, zb = gpu.qr_preprocess(Hb, y)
    Rb[4, r_off_level(n, 3) + 1] = float("inf")  # row of level 3, column 4: met only at level 3
    zb[7, n - 1] = float("nan")                     # the top level
    got = [_np(t) for t in run(Rb, zb)]
    sym, pd, flags, ctr = got
    for b in (1, 4, 7):
        assert flags[b] == gpu.FLAG_NONFINITE_INPUT, (variant, b, flags[b])
        assert np.all(sym[b] == 0) and np.isinf(pd[b])
    if not variant.startswith("hybrid"):
        assert ctr[7, 0] == 0 and 0 < ctr[4, 0] < clean[3][4, 0]  # frame 4 stopped at level 3
    keep = np.setdiff1d(np.arange(B), [1, 4, 7])
    for a, c in zip(got, clean):
        assert np.array_equal(a[keep], c[keep]), variant


def r_off_level(n, k):
    return (n - 1 - k) * (n - k) // 2


@pytest.mark.parametrize("variant", ["register", "two frames per wave", "survivor lists in LDS", "complex levels"])
def test_empty_sphere_rerun_all_variants(gpu, orc, variant):
    """A radius below every frame's leaf: each kernel variant detects the
    frame again without a radius, equal (symbols, pd) to the unbounded run,
    with flags EMPTY_SPHERE | FOUND and counters summing both searches."""
    import torch

    M, q, K = {"register": (16, 16, 16), "two frames per wave": (40, 64, 4),
               "survivor lists in LDS": (8, 16, 128), "complex levels": (16, 64, 10)}[variant]
    B, P = 9, math.isqrt(q)
    f = gen_frames(M, M, q, 14.0, B, seed=2950 + M)
    H, y, _ = _dev(f)
    R, z = gpu.qr_preprocess(H, y)
    fn = gpu.kbest_detect_complex if variant == "complex levels" else gpu.kbest_detect
    print(f"empty-sphere re-run {variant}", flush=True)
    s0, p0, f0, c0 = [_np(t) for t in fn(R, z, M, P, K, want_counters=True)]
    r2 = torch.from_numpy((p0 * 0.05).astype(np.float32)).cuda()
    r2[0] = float(p0[0]) * 4.0  # frame 0 keeps its leaf inside the sphere
    s1, p1, f1, c1 = [_np(t) for t in fn(R, z, M, P, K, radius2=r2, want_counters=True)]
    assert f1[0] == gpu.FLAG_FOUND and np.array_equal(s1[0], s0[0])
    assert np.all(f1[1:] == gpu.FLAG_FOUND | gpu.FLAG_EMPTY_SPHERE)
    if variant == "two frames per wave":
        # the re-run takes the one-frame kernel, which sums a centre over eight
        # lanes instead of four: equal up to FP32 rounding of the pd
        assert np.allclose(p1, p0, rtol=1e-5)
        assert np.all(np.all(s1 == s0, axis=1) | (np.abs(p1 - p0) <= 1e-5 * p0))
    else:
        assert np.array_equal(s1, s0) and np.array_equal(p1, p0)
    assert np.all(c1[1:, 0] > c0[1:, 0]) and np.all(c1[1:, 0] < 2 * c0[1:, 0] + 1)


def test_kbest_scheduled_near_singular_channel(gpu, orc):
    """Scheduled 64-QAM K-best with a cap of 16 survivors (the row-recompute
    kernel with two blocks of candidates) on channels with two nearly
    parallel column pairs: at the small diagonal entries' levels most
    candidates fall below the bound, so the second compaction of
    kb_select_bounded and the sort of every block both run."""
    import torch

    M, q, B, K = 12, 64, 40, 16
    P = math.isqrt(q)
    f = gen_frames(M, M, q, 24.0, B, seed=9910)
    rng = np.random.default_rng(9911)
    H = f.H.copy()
    for c in (4, 9):
        d = (rng.standard_normal((B, M)) + 1j * rng.standard_normal((B, M))) / np.sqrt(2)
        H[:, :, c] = (H[:, :, c - 1] + 0.05 * d).astype(np.complex64)
    sched = rng.integers(9, K + 1, (B, 2 * M)).astype(np.int32)
    print(f"scheduled K-best near-singular {M}x{M} {q}-QAM B={B} cap {K}", flush=True)
    R, z = gpu.qr_preprocess(torch.from_numpy(H).cuda(), torch.from_numpy(f.y).cuda())
    sym, pd, flags, ctr = gpu.kbest_detect(R, z, M, P, K, k_sched=torch.from_numpy(sched).cuda(),
                                           want_counters=True)
    Ro, zo, _ = orc.qr(H, f.y)
    out = orc.kbest(Ro, zo, P, K, k_sched=sched)
    _, tol, _ = check_kbest_run(orc, "scheduled near-singular", P, K, _np(sym), _np(pd), out, Ro, zo, k_sched=sched)
    clean = out["margin"][:, 0] > tol
    assert np.array_equal(_np(ctr)[clean, :2], out["counters"][clean, :2])

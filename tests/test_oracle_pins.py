"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties one oracle routine to something other than itself: brute
force on tiny systems, closed forms, special cases that reduce to textbook
routines, library routines and the node counts the paper prints.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2002_09561_amd.framegen import gen_frames, qam_amplitudes

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def real_model_np(H, y):
    """Real representation written with numpy block assignments."""
    B, N, M = H.shape
    Hr = np.zeros((B, 2 * N, 2 * M))
    Hr[:, 0::2, 0::2] = H.real
    Hr[:, 0::2, 1::2] = -H.imag
    Hr[:, 1::2, 0::2] = H.imag
    Hr[:, 1::2, 1::2] = H.real
    yr = np.zeros((B, 2 * N))
    yr[:, 0::2] = y.real
    yr[:, 1::2] = y.imag
    return Hr, yr


# --------------------------------------------------------------- frames
def test_frames_unit_energy_and_noise():
    for q in (4, 16, 64):
        a = qam_amplitudes(q)
        # E|s|^2 over the square constellation is exactly 1
        e = np.mean(np.add.outer(a ** 2, a ** 2))
        assert abs(e - 1.0) < 1e-14
    f = gen_frames(8, 8, 16, 10.0, 4000, seed=3)
    amp = qam_amplitudes(16)
    s = amp[f.s_idx // 4] + 1j * amp[f.s_idx % 4]
    n = f.y.astype(np.complex128) - np.einsum("bij,bj->bi", f.H.astype(np.complex128), s)
    assert abs(np.mean(np.abs(n) ** 2) / f.sigma2 - 1.0) < 0.03
    assert abs(np.mean(np.abs(f.H) ** 2) - 1.0) < 0.02
    g = gen_frames(8, 8, 16, 10.0, 10, seed=3)
    assert np.array_equal(g.H, f.H[:10]) and np.array_equal(g.y, f.y[:10])


# --------------------------------------------------------------- QR (Sec. III-B)
@pytest.mark.parametrize("N,M,q", [(4, 4, 4), (6, 4, 16), (16, 16, 16), (12, 7, 64)])
def test_qr_properties(orc, N, M, q):
    f = gen_frames(N, M, q, 15.0, 20, seed=N * 100 + M)
    R, z, resid = orc.qr(f.H, f.y)
    Hr, yr = real_model_np(f.H.astype(np.complex128), f.y.astype(np.complex128))
    n = 2 * M
    for b in range(len(f)):
        assert np.allclose(np.tril(R[b], -1), 0.0)
        assert np.all(np.diag(R[b]) > 0)
        # R^T R = H_r^T H_r and H_r^T y_r = R^T z
        assert np.allclose(R[b].T @ R[b], Hr[b].T @ Hr[b], atol=1e-10)
        assert np.allclose(Hr[b].T @ yr[b], R[b].T @ z[b], atol=1e-10)
        # Q = H_r R^-1 has orthonormal columns
        Q = Hr[b] @ np.linalg.inv(R[b])
        assert np.allclose(Q.T @ Q, np.eye(n), atol=1e-9)
        # library QR up to row signs
        Rl = np.linalg.qr(Hr[b], mode="r")
        sg = np.sign(np.diag(Rl))
        assert np.allclose(sg[:, None] * Rl, R[b], atol=1e-10)
        # interleaved block structure of the complex QR
        assert np.allclose(R[b][np.arange(0, n, 2), np.arange(1, n, 2)], 0.0, atol=1e-12)
        assert np.allclose(R[b][np.arange(0, n, 2), np.arange(0, n, 2)],
                           R[b][np.arange(1, n, 2), np.arange(1, n, 2)], atol=1e-12)
        # residual ||y||^2 - ||z||^2
        assert abs(resid[b] - (yr[b] @ yr[b] - z[b] @ z[b])) < 1e-9 * (yr[b] @ yr[b])
        if N == M:
            assert resid[b] == 0.0


# --------------------------------------------------------------- Eq. (2) brute force
def test_bruteforce_noiseless_returns_truth(orc):
    f = gen_frames(3, 3, 16, 300.0, 30, seed=9)
    s, m = orc.brute_force(f.H, f.y, 16)
    assert np.array_equal(s, f.s_idx)
    assert np.all(m < 1e-9)


def test_bruteforce_is_minimum_over_random_candidates(orc):
    f = gen_frames(3, 3, 16, 5.0, 40, seed=10)
    s, m = orc.brute_force(f.H, f.y, 16)
    rng = np.random.default_rng(0)
    for _ in range(20):
        cand = rng.integers(0, 16, size=s.shape).astype(np.int32)
        assert np.all(orc.metric(f.H, f.y, cand, 16) >= m - 1e-12)
    # the metric of the truth is never below the ML metric
    assert np.all(orc.metric(f.H, f.y, f.s_idx, 16) >= m - 1e-12)


# --------------------------------------------------------------- T1: SD == ML
@pytest.mark.parametrize("N,M,q,snr,B", [(4, 4, 4, 10.0, 1000), (3, 3, 16, 8.0, 150),
                                         (4, 3, 16, 4.0, 100), (2, 2, 64, 12.0, 100)])
def test_sesd_equals_bruteforce(orc, N, M, q, snr, B):
    f = gen_frames(N, M, q, snr, B, seed=11 + M)
    P = math.isqrt(q)
    R, z, resid = orc.qr(f.H, f.y)
    sb, mb = orc.brute_force(f.H, f.y, q)
    x, pd, fl, ctr = orc.sesd(R, z, P)
    assert np.all(fl & orc.CERTIFIED)
    assert np.array_equal(orc.x_to_sym(x, P), sb)
    # T6: the leaf pd equals ||y - Hs||^2 minus the constant residual
    assert np.allclose(pd + resid, mb, rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------- T2: K-best with full K == ML
def test_kbest_full_K_equals_bruteforce(orc):
    f = gen_frames(4, 4, 4, 6.0, 300, seed=21)
    R, z, _ = orc.qr(f.H, f.y)
    sb, _ = orc.brute_force(f.H, f.y, 4)
    out = orc.kbest(R, z, 2, 2 ** 7)
    assert np.array_equal(orc.x_to_sym(out["x"], 2), sb)
    f = gen_frames(2, 2, 16, 3.0, 100, seed=22)
    R, z, _ = orc.qr(f.H, f.y)
    sb, _ = orc.brute_force(f.H, f.y, 16)
    out = orc.kbest(R, z, 4, 4 ** 3)
    assert np.array_equal(orc.x_to_sym(out["x"], 4), sb)


# --------------------------------------------------------------- T3/T4: K=1 == SIC == first SD leaf
@pytest.mark.parametrize("M,q", [(4, 4), (16, 16), (32, 64)])
def test_k1_and_first_sd_leaf_equal_sic(orc, M, q):
    f = gen_frames(M, M, q, 14.0, 50, seed=30 + M)
    P = math.isqrt(q)
    R, z, _ = orc.qr(f.H, f.y)
    xs, pds = orc.zf_sic(R, z, P)
    k1 = orc.kbest(R, z, P, 1)
    assert np.array_equal(k1["x"], xs)
    assert np.allclose(k1["pd"], pds, rtol=1e-12)
    # Best-FS reaches its first leaf after exactly n expansions, straight down
    x, pd, fl, ctr = orc.sesd(R, z, P, budget=2 * M)
    assert np.array_equal(x, xs)
    assert np.all(ctr[:, 0] == 2 * M)


# --------------------------------------------------------------- T5/T6 on K-best leaves
def test_pd_terms_monotone_and_leaf_identity(orc):
    f = gen_frames(10, 8, 16, 10.0, 30, seed=40)
    R, z, resid = orc.qr(f.H, f.y)
    out = orc.kbest(R, z, 4, 8)
    m = orc.metric(f.H, f.y, orc.x_to_sym(out["x"], 4), 16)
    for b in range(len(f)):
        g = orc.path_terms(R[b], z[b], out["x"][b], 4)
        assert np.all(g >= 0.0)
        cum = np.cumsum(g[::-1])
        assert np.all(np.diff(cum) >= 0.0)
        assert abs(cum[-1] - out["pd"][b]) < 1e-9 * max(1.0, cum[-1])
        assert abs(cum[-1] + resid[b] - m[b]) < 1e-9 * max(1.0, m[b])


# --------------------------------------------------------------- T8: node counts
def test_kbest_node_counts_real_levels(orc):
    f = gen_frames(8, 8, 16, 10.0, 5, seed=50)
    R, z, _ = orc.qr(f.H, f.y)
    n, P = 16, 4
    for K in (1, 3, 16, 64):
        out = orc.kbest(R, z, P, K)
        expect = sum(min(K, P ** t) for t in range(n))
        assert np.all(out["counters"][:, 0] == expect)
        assert np.all(out["counters"][:, 1] == P * expect)


def test_kbest_node_counts_match_paper_figure(orc):
    """Complex-symbol K-best (J = 2 real levels per step) visits the node
    counts printed in the paper for 16x16 64-QAM."""
    path = __file__.replace("test_oracle_pins.py", "golden/kbest_visited_nodes.txt")
    rows = [list(map(int, l.split())) for l in open(path) if l.strip() and not l.startswith("#")]
    for M, q, K, visited in rows:
        f = gen_frames(M, M, q, 20.0, 3, seed=51)
        R, z, _ = orc.qr(f.H, f.y)
        out = orc.kbest(R, z, math.isqrt(q), K, J=2)
        assert np.all(out["counters"][:, 0] == visited)


# --------------------------------------------------------------- radius
def test_kbest_radius(orc):
    f = gen_frames(8, 8, 16, 10.0, 40, seed=60)
    R, z, _ = orc.qr(f.H, f.y)
    ml = orc.sesd(R, z, 4)
    r2 = float(np.median(ml[1])) * 1.5
    out = orc.kbest(R, z, 4, 16, r2=r2)
    free = orc.kbest(R, z, 4, 16)
    inside = (out["flags"] & orc.EMPTY_SPHERE) == 0
    assert np.all(out["flags"] & orc.FOUND)
    assert np.all(out["pd"][inside] < r2)
    assert (~inside).any() and np.array_equal(out["x"][~inside], free["x"][~inside])
    # a radius below the ML metric leaves nothing inside the sphere: every
    # frame is searched again without a radius
    tiny = orc.kbest(R, z, 4, 16, r2=float(ml[1].min()) * 0.5)
    assert np.all(tiny["flags"] & orc.EMPTY_SPHERE) and np.all(tiny["flags"] & orc.FOUND)
    assert np.array_equal(tiny["x"], free["x"])
    sd = orc.sesd(R, z, 4, r2=np.full(len(f), float(ml[1].min()) * 0.5))
    assert np.all(sd[2] & orc.EMPTY_SPHERE) and np.array_equal(sd[0], ml[0])


def test_sesd_warm_start(orc):
    f = gen_frames(16, 16, 16, 8.0, 20, seed=61)
    R, z, _ = orc.qr(f.H, f.y)
    kb = orc.kbest(R, z, 4, 16)
    ref = orc.sesd(R, z, 4)
    warm = orc.sesd(R, z, 4, r2=kb["pd"] * (1 + 1e-12), x_init=kb["x"])
    assert np.array_equal(warm[0], ref[0])
    assert np.all(warm[2] & orc.CERTIFIED)
    assert np.all(warm[3][:, 0] <= ref[3][:, 0])


# --------------------------------------------------------------- T9: hybrid special cases
def test_hybrid_degenerate_cases(orc):
    f = gen_frames(4, 4, 16, 8.0, 120, seed=70)
    R, z, _ = orc.qr(f.H, f.y)
    sb, _ = orc.brute_force(f.H, f.y, 16)
    h0 = orc.hybrid(R, z, 4, 0, 1)
    assert np.array_equal(orc.x_to_sym(h0["x"], 4), sb)
    for Kw in (1, 3, 8):
        hm = orc.hybrid(R, z, 4, 1, Kw, master_off=True)
        kb = orc.kbest(R, z, 4, Kw)
        assert np.array_equal(hm["x"], kb["x"])
    hf = orc.hybrid(R, z, 4, 3, 4 ** 7)
    assert np.array_equal(orc.x_to_sym(hf["x"], 4), sb)


def test_hybrid_never_beats_ml(orc):
    f = gen_frames(12, 12, 16, 6.0, 40, seed=71)
    R, z, _ = orc.qr(f.H, f.y)
    ml = orc.sesd(R, z, 4)
    for W, Kw in ((1, 1), (4, 2), (19, 8)):
        h = orc.hybrid(R, z, 4, W, Kw)
        assert np.all(h["pd"] >= ml[1] * (1 - 1e-12))
        assert np.all(h["flags"] & orc.FOUND)


def test_hybrid_tracks_at_least_the_sic_leaf(orc):
    """The master reaches the SIC leaf first (Best-FS), so the hybrid is never
    worse than SIC; with more workers it gets at least as close to ML on
    average."""
    f = gen_frames(16, 16, 64, 18.0, 60, seed=72)
    R, z, _ = orc.qr(f.H, f.y)
    _, pds = orc.zf_sic(R, z, 8)
    h = orc.hybrid(R, z, 8, 4, 2, budget=20000)
    assert np.all(h["pd"] <= pds * (1 + 1e-12))


# --------------------------------------------------------------- learned-pruning state and labels
def test_prune_features_noiseless(orc):
    f = gen_frames(6, 6, 16, 300.0, 10, seed=80)
    R, z, _ = orc.qr(f.H, f.y)
    feat = orc.prune_features(R, z, 4, 1e-4)
    n = 12
    assert np.allclose(feat[:, :, 0], np.arange(n) / n)
    # the SIC centre sits on the transmitted point: one half spacing from
    # the nearest decision boundary, and no accumulated distance
    assert np.allclose(feat[:, :, 1], 0.5, atol=1e-9)
    assert np.allclose(feat[:, :, 3], 0.0, atol=1e-9)
    c = orc.pam_scale(4)
    sr = math.sqrt(1e-4 / 2)
    assert np.allclose(feat[:, :, 2], np.log2(np.diagonal(R, axis1=1, axis2=2) * 2 * c / sr))


def test_forced_rank_labels_brute_force(orc):
    """Rank of the ML prefix among all children of all prefixes, by
    enumeration, equals the label the forced K-best reports when K keeps
    every prefix."""
    f = gen_frames(2, 2, 16, 4.0, 15, seed=81)
    R, z, _ = orc.qr(f.H, f.y)
    P, n = 4, 4
    ml = orc.sesd(R, z, P)[0]
    out = orc.kbest(R, z, P, P ** n, force_path=ml)
    amp = orc.amplitudes(P)
    for b in range(len(f)):
        for t in range(n):
            k = n - 1 - t
            levels = list(range(n - 1, k - 1, -1))

            def pd_of(assign):
                s = 0.0
                for kk in levels:
                    e = z[b, kk] - sum(R[b, kk, j] * amp[assign[j]] for j in range(kk, n))
                    s += e * e
                return s

            target = pd_of({j: ml[b, j] for j in levels})
            smaller = 0
            for combo in itertools.product(range(P), repeat=len(levels)):
                if pd_of(dict(zip(levels, combo))) < target:
                    smaller += 1
            assert out["rank"][b, k] == smaller + 1
    assert np.array_equal(out["x"], ml)
    # with K = 1 and the SIC path forced, the forced prefix is always first
    xs, _ = orc.zf_sic(R, z, P)
    o1 = orc.kbest(R, z, P, 1, force_path=xs)
    assert np.all(o1["rank"] == 1)


# --------------------------------------------------------------- T10: MLP
def _mlp_params(orc, seed):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.3, orc.MLP_NPARAM)
    return w


def test_mlp_forward_matches_matrix_form(orc):
    w = _mlp_params(orc, 0)
    X = np.random.default_rng(1).normal(size=(50, 4))
    H = orc.MLP_H
    o = 0
    W1 = w[o:o + H * 4].reshape(H, 4); o += H * 4
    b1 = w[o:o + H]; o += H
    W2 = w[o:o + H * H].reshape(H, H); o += H * H
    b2 = w[o:o + H]; o += H
    w3 = w[o:o + H]; o += H
    b3 = w[o]
    ref = np.maximum(np.maximum(X @ W1.T + b1, 0) @ W2.T + b2, 0) @ w3 + b3
    assert np.allclose(orc.mlp_forward(w, X), ref, rtol=1e-12, atol=1e-12)


def test_mlp_gradient_finite_differences(orc):
    w = _mlp_params(orc, 2)
    rng = np.random.default_rng(3)
    X = rng.normal(size=(16, 4))
    y = rng.normal(size=16) * 3
    loss, g = orc.mlp_loss_grad(w, X, y, 0.95)
    h = 1e-6
    idx = list(rng.choice(orc.MLP_NPARAM, 60, replace=False)) + [orc.MLP_NPARAM - 1, 0, 600]
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (orc.mlp_loss_grad(wp, X, y, 0.95)[0] - orc.mlp_loss_grad(wm, X, y, 0.95)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])


def test_pinball_loss_closed_form(orc):
    w = np.zeros(orc.MLP_NPARAM)
    w[-1] = 1.0  # constant output 1
    X = np.zeros((4, 4))
    y = np.array([3.0, 0.0, 1.5, -1.0])
    loss, g = orc.mlp_loss_grad(w, X, y, 0.9)
    # residuals 2, -1, 0.5, -2 -> 0.9*2 + 0.1*1 + 0.9*0.5 + 0.1*2
    assert abs(loss - (1.8 + 0.1 + 0.45 + 0.2) / 4) < 1e-15
    assert abs(g[-1] - (-0.9 + 0.1 - 0.9 + 0.1) / 4) < 1e-15


def test_adam_first_step_is_signed_lr(orc):
    rng = np.random.default_rng(4)
    w = rng.normal(size=100)
    g = rng.normal(size=100)
    m = np.zeros(100)
    v = np.zeros(100)
    w0 = w.copy()
    orc.adam_step(w, m, v, g, 1, 1e-2, eps=0.0)
    assert np.allclose(w0 - w, 1e-2 * np.sign(g), rtol=1e-12)


# --------------------------------------------------------------- T11: Gray map
@pytest.mark.parametrize("P", [2, 4, 8])
def test_gray_adjacent_points_differ_in_one_bit(orc, P):
    s = np.arange(P * P)
    bits = orc.gray_bits(s, P)
    for a in range(P * P):
        for b in range(P * P):
            ia, ja, ib, jb = a // P, a % P, b // P, b % P
            if abs(ia - ib) + abs(ja - jb) == 1:
                assert (bits[a] != bits[b]).sum() == 1
    assert len({tuple(r) for r in bits}) == P * P


# --------------------------------------------------------------- linear baselines and the paper's radius
def _slice_np(u, P):
    c = math.sqrt(3.0 / (2.0 * (P * P - 1)))
    return np.clip(np.floor((u / c + (P - 1)) / 2.0 + 0.5), 0, P - 1).astype(np.int32)


@pytest.mark.parametrize("N,M,q", [(6, 6, 16), (8, 5, 64)])
def test_linear_zf_equals_least_squares(orc, N, M, q):
    """Back-substitution on the plain QR is the least-squares (zero-forcing)
    solution; checked against numpy's lstsq on the complex system."""
    P = math.isqrt(q)
    f = gen_frames(N, M, q, 12.0, 40, seed=41 + N)
    R, z, _ = orc.qr(f.H, f.y)
    x, u = orc.linear(R, z, P)
    for b in range(len(f)):
        s = np.linalg.lstsq(f.H[b].astype(np.complex128), f.y[b].astype(np.complex128), rcond=None)[0]
        ur = np.stack([s.real, s.imag], -1).reshape(-1)
        assert np.allclose(u[b], ur, atol=1e-10)
        assert np.array_equal(x[b], _slice_np(ur, P))


def test_mmse_qr_normal_equations(orc):
    f = gen_frames(7, 5, 16, 6.0, 20, seed=5)
    R, z = orc.qr_mmse(f.H, f.y, f.sigma2)
    Hr, yr = real_model_np(f.H.astype(np.complex128), f.y.astype(np.complex128))
    n = 10
    for b in range(len(f)):
        assert np.allclose(np.tril(R[b], -1), 0.0) and np.all(np.diag(R[b]) > 0)
        assert np.allclose(R[b].T @ R[b], Hr[b].T @ Hr[b] + f.sigma2 * np.eye(n), atol=1e-10)
        assert np.allclose(R[b].T @ z[b], Hr[b].T @ yr[b], atol=1e-10)


def test_linear_mmse_equals_regularised_solve(orc):
    P = 4
    f = gen_frames(8, 8, 16, 8.0, 40, seed=17)
    R, z = orc.qr_mmse(f.H, f.y, f.sigma2)
    x, u = orc.linear(R, z, P)
    for b in range(len(f)):
        H = f.H[b].astype(np.complex128)
        s = np.linalg.solve(H.conj().T @ H + f.sigma2 * np.eye(8), H.conj().T @ f.y[b].astype(np.complex128))
        ur = np.stack([s.real, s.imag], -1).reshape(-1)
        assert np.allclose(u[b], ur, atol=1e-10)
        assert np.array_equal(x[b], _slice_np(ur, P))


def test_mmse_limits(orc):
    """sigma2 -> 0 gives the plain QR (zero forcing); on noiseless frames the
    MMSE-SIC leaf (K = 1 on the MMSE QR) with a tiny load is the truth."""
    f = gen_frames(6, 6, 64, 100.0, 30, seed=9)
    R0, z0, _ = orc.qr(f.H, f.y)
    R1, z1 = orc.qr_mmse(f.H, f.y, 1e-14)
    assert np.allclose(R1, R0, atol=1e-6) and np.allclose(z1, z0, atol=1e-6)
    amp = qam_amplitudes(64)
    s = (amp[f.s_idx // 8] + 1j * amp[f.s_idx % 8]).astype(np.complex64)
    y0 = np.einsum("bij,bj->bi", f.H, s).astype(np.complex64)
    Rm, zm = orc.qr_mmse(f.H, y0, 1e-6)
    out = orc.kbest(Rm, zm, 8, 1)
    assert np.array_equal(orc.x_to_sym(out["x"], 8), f.s_idx)


def test_mrc_orthogonal_channel_is_exact(orc):
    """With orthogonal columns, matched filtering decouples the streams:
    MRC equals zero forcing, and on noiseless frames it returns the truth."""
    rng = np.random.default_rng(4)
    B, N, M, q = 10, 8, 5, 16
    H = np.empty((B, N, M), np.complex64)
    for b in range(B):
        Q, _ = np.linalg.qr(rng.standard_normal((N, M)) + 1j * rng.standard_normal((N, M)))
        H[b] = (Q * rng.uniform(0.5, 2.0, M)).astype(np.complex64)
    s_idx = rng.integers(0, q, (B, M)).astype(np.int32)
    amp = qam_amplitudes(q)
    s = amp[s_idx // 4] + 1j * amp[s_idx % 4]
    y = np.einsum("bij,bj->bi", H.astype(np.complex128), s).astype(np.complex64)
    sm, um = orc.mrc(H, y, q)
    assert np.array_equal(sm, s_idx)
    R, z, _ = orc.qr(H, y)
    _, uz = orc.linear(R, z, 4)
    assert np.allclose(um, uz, atol=1e-5)


def test_paper_radius_keeps_ml_when_inside(orc):
    """With the paper's radius r^2 = N M sigma^2 (squared, Sec. IV), the
    radius-limited SD returns the ML vector on every frame whose ML metric
    lies inside the sphere.  That radius is M times the expected noise energy
    N sigma^2, so at this size every ML metric lies inside; a sphere half as
    large as the smallest ML metric is empty on every frame."""
    N = M = 6
    f = gen_frames(N, M, 16, 4.0, 60, seed=23)
    R, z, resid = orc.qr(f.H, f.y)
    xs, pd_inf, _, _ = orc.sesd(R, z, 4)
    r2 = np.full(len(f), N * M * f.sigma2)
    xr, pd_r, fl, _ = orc.sesd(R, z, 4, r2=r2)
    assert np.all(pd_inf < r2)
    assert np.array_equal(xr, xs) and np.allclose(pd_r, pd_inf)
    x0, _, fl0, _ = orc.sesd(R, z, 4, r2=np.full(len(f), 0.5 * pd_inf.min()))
    assert np.all((fl0 & orc.EMPTY_SPHERE) != 0) and np.array_equal(x0, xs)


# --------------------------------------------------------------- hybrid round schedule (Sec. VI)
_TRACE_RT = np.array([[1, 0, 0.5, 0.5], [0, 1, 0.5, 0], [0, 0, 1, 0.5], [0, 0, 0, 1.0]])
_TRACE_Z = np.array([0.1, 0.2, -0.1, 0.3])


def test_hybrid_round_schedule_golden_trace(orc):
    """The deterministic-round reading of the SD-K-best master/worker scheme
    traced by hand on a 4-level tree (derivation in the golden file): pool
    contents, hand-offs, worker levels, candidates, radius updates and the
    final counters.  Each of these oracle mutations changes the trace while
    leaving the detected symbols unchanged: workers taking a node while the
    pool holds a single one (pool >= 1), the master expanding a node already
    outside the sphere instead of discarding it, and workers taking the
    left-most node instead of the right-most."""
    path = __file__.replace("test_oracle_pins.py", "golden/hybrid_trace_2x2_4qam_w2_k1.txt")
    gold = [l for l in open(path).read().splitlines() if l and not l.startswith("#")]
    c = orc.pam_scale(2)
    lines, x, pd, fl, ctr = orc.hybrid_trace(_TRACE_RT / c, _TRACE_Z, 2, 2, 1)
    assert lines == gold
    assert list(x) == [1, 1, 0, 1] and abs(pd - 1.55) < 1e-12
    assert list(ctr) == [9, 18, 5, 1] and (fl & orc.CERTIFIED) and (fl & orc.FOUND)
    # the batched driver runs the same schedule
    h = orc.hybrid((_TRACE_RT / c)[None], _TRACE_Z[None], 2, 2, 1)
    assert list(h["x"][0]) == [1, 1, 0, 1] and list(h["counters"][0]) == [9, 18, 5, 1]


def test_hybrid_complex_levels_golden_trace(orc):
    """The hybrid with J = 2 real levels per step (one complex symbol, P^2
    children) on the frame of the real-level trace, traced by hand (the
    derivation is in the golden file).  It fails if a child's digits are
    stored with the lower level first, if the lower level's centre misses
    the step's own upper symbol, if leaves are detected one level early, or
    if a child counts one evaluation instead of J."""
    path = __file__.replace("test_oracle_pins.py", "golden/hybrid_trace_2x2_4qam_j2_w1_k1.txt")
    gold = [l for l in open(path).read().splitlines() if l and not l.startswith("#")]
    c = orc.pam_scale(2)
    lines, x, pd, fl, ctr = orc.hybrid_trace(_TRACE_RT / c, _TRACE_Z, 2, 1, 1, J=2)
    assert lines == gold
    assert list(x) == [1, 1, 0, 1] and abs(pd - 1.55) < 1e-12
    assert list(ctr) == [4, 32, 3, 1] and (fl & orc.CERTIFIED) and (fl & orc.FOUND)
    h = orc.hybrid((_TRACE_RT / c)[None], _TRACE_Z[None], 2, 1, 1, J=2)
    assert list(h["x"][0]) == [1, 1, 0, 1] and list(h["counters"][0]) == [4, 32, 3, 1]


@pytest.mark.parametrize("M,q,snr", [(2, 16, 4.0), (3, 4, 2.0), (2, 64, 12.0)])
def test_hybrid_complex_levels_special_cases(orc, M, q, snr):
    """J = 2: with no workers the master alone is an exact SD (the brute-force
    ML metric); with the master off, worker 0 runs the complex-level K-best
    (orc.kbest with J = 2: the same points and node counters)."""
    from paper_2002_09561_amd.framegen import gen_frames

    f = gen_frames(M, M, q, snr, 40, seed=77 + M)
    R, z, _ = orc.qr(f.H, f.y)
    P = math.isqrt(q)
    h = orc.hybrid(R, z, P, 0, 1, J=2)
    assert np.all(h["flags"] & orc.CERTIFIED)
    s_bf, _ = orc.brute_force(f.H, f.y, q)
    mh = orc.metric(f.H, f.y, orc.x_to_sym(h["x"], P), q)
    mb = orc.metric(f.H, f.y, s_bf, q)
    assert np.allclose(mh, mb, rtol=1e-12)
    for K in (1, 3, 8):
        hk = orc.hybrid(R, z, P, 1, K, master_off=True, J=2)
        kb = orc.kbest(R, z, P, K, J=2)
        assert np.array_equal(hk["x"], kb["x"])
        assert np.array_equal(hk["counters"][:, :2], kb["counters"][:, :2])


def test_hybrid_trace_no_workers_is_best_first_sd(orc):
    """With no workers the trace is the Best-FS SD of Alg. 1 on the same
    tree: the master alone walks down the best children (0.49, 0.65, 0.74,
    leaf 1.55), then pops the remaining siblings, each either outside the
    sphere (stale) or expanded into leaves above the radius."""
    c = orc.pam_scale(2)
    lines, x, pd, fl, ctr = orc.hybrid_trace(_TRACE_RT / c, _TRACE_Z, 2, 0, 1)
    assert list(x) == [1, 1, 0, 1] and abs(pd - 1.55) < 1e-12
    assert lines[:3] == ["round 1 r2 inf pool 1", "master expand depth 0 pd 0", "  child 1 pd 0.49"]
    assert "radius 1.55 from source 0" in lines
    assert not any(l.startswith("worker") for l in lines)
    # every pop after the radius fell to 1.55 lies above it: the siblings
    # 1.69 (depth 1), 3.05 (depth 2) and 3.54 (depth 3) are discarded
    stale = sorted(l for l in lines if "stale" in l and l.startswith("master"))
    assert stale == ["master stale depth 1 pd 1.69", "master stale depth 2 pd 3.05", "master stale depth 3 pd 3.54"]
    sd = orc.sesd((_TRACE_RT / c)[None], _TRACE_Z[None], 2)
    assert list(sd[0][0]) == [1, 1, 0, 1] and ctr[0] == sd[3][0, 0]


# --------------------------------------------------------------- near-tie margins
def _two_level(rt, z, P=2):
    c = orc_scale = math.sqrt(3.0 / (2.0 * (P * P - 1)))
    return np.asarray(rt, float)[None] / orc_scale, np.asarray(z, float)[None]


def test_kbest_margin_exact_tie(orc):
    """z = 0 on an identity R: both children of every node have the same pd,
    so the K = 1 selection (and the final choice) is an exact tie: margin 0
    between two equal keys; the tie rule keeps child 0."""
    R, z = _two_level([[1, 0], [0, 1]], [0.0, 0.0])
    out = orc.kbest(R, z, 2, 1)
    assert out["margin"][0, 0] == 0.0
    assert out["margin"][0, 1] == out["margin"][0, 2] == pytest.approx(1.0)
    assert list(out["x"][0]) == [0, 0]


def test_kbest_margin_known_gap(orc):
    """Level 1: e = 0.1 - v gives 0.81 (v = +1) and 1.21 (v = -1), a relative
    gap of 0.4 / 1.21 at the K = 1 boundary; level 0 from 0.81: e = 0.5 - v
    gives 1.06 and 3.06 (gap 2 / 3.06).  The smaller gap is returned with its
    pair (kept key, first dropped key)."""
    R, z = _two_level([[1, 0], [0, 1]], [0.5, 0.1])
    out = orc.kbest(R, z, 2, 1)
    assert out["margin"][0, 0] == pytest.approx(0.4 / 1.21, rel=1e-12)
    assert out["margin"][0, 1] == pytest.approx(0.81) and out["margin"][0, 2] == pytest.approx(1.21)
    assert out["pd"][0] == pytest.approx(1.06)


def test_kbest_margin_radius_test(orc):
    """With r2 = 1.07 the radius test of the leaf 1.06 is the closest
    decision: relative gap 0.01 / 1.07 between the leaf and the radius (the
    other children lie outside the sphere by wider gaps and no selection is
    left to make)."""
    R, z = _two_level([[1, 0], [0, 1]], [0.5, 0.1])
    out = orc.kbest(R, z, 2, 1, r2=1.07)
    assert out["margin"][0, 0] == pytest.approx(0.01 / 1.07, rel=1e-9)
    assert out["margin"][0, 1] == pytest.approx(1.06) and out["margin"][0, 2] == pytest.approx(1.07)
    assert (out["flags"][0] & orc.FOUND) and not (out["flags"][0] & orc.EMPTY_SPHERE)


def test_empty_sphere_is_searched_again_without_radius(orc):
    """A radius below every leaf (r2 = 1.0 < 1.06 here) leaves the sphere
    empty; the reading searches the frame again with r2 = +inf: the result is
    that of the unbounded search, the flags keep EMPTY_SPHERE next to FOUND,
    and the counters add up both searches (one root and one level-1 node in
    the first, as in the second)."""
    R, z = _two_level([[1, 0], [0, 1]], [0.5, 0.1])
    free = orc.kbest(R, z, 2, 1)
    out = orc.kbest(R, z, 2, 1, r2=1.0)
    assert (out["flags"][0] & orc.EMPTY_SPHERE) and (out["flags"][0] & orc.FOUND)
    assert np.array_equal(out["x"], free["x"]) and out["pd"][0] == free["pd"][0]
    assert out["counters"][0, 0] == 2 * free["counters"][0, 0]
    # the radius test 0.81 < 1.0 < 1.06 is the closest decision of the first search
    assert out["margin"][0, 0] == pytest.approx(0.06 / 1.06, rel=1e-9)
    sd = orc.sesd(R, z, 2, r2=np.array([1.0]))
    assert (sd[2][0] & orc.EMPTY_SPHERE) and (sd[2][0] & orc.FOUND) and list(sd[0][0]) == list(free["x"][0])
    h = orc.hybrid(R, z, 2, 1, 1, r2=1.0)
    assert (h["flags"][0] & orc.EMPTY_SPHERE) and list(h["x"][0]) == list(free["x"][0])


def test_forced_path_gap(orc):
    """Forcing the other child at level 1 (v = -1, pd 1.21 against the kept
    0.81) gives the gap of the decision that dropped it; forcing the search's
    own path gives 0.  At the leaves, forcing the second-best leaf of the
    kept survivor (3.06 against 1.06) gives that final gap."""
    R, z = _two_level([[1, 0], [0, 1]], [0.5, 0.1])
    own = orc.kbest(R, z, 2, 1)
    o0 = orc.kbest(R, z, 2, 1, force_path=own["x"])
    assert o0["fgap"][0] == 0.0
    o1 = orc.kbest(R, z, 2, 2, force_path=np.array([[0, 1]], np.int32))
    assert o1["fgap"][0] == pytest.approx(2.0 / 3.06, rel=1e-12)  # leaf 3.06 vs best leaf 1.06
    o2 = orc.kbest(R, z, 2, 1, force_path=np.array([[1, 0]], np.int32))
    assert o2["fgap"][0] >= 0.4 / 1.21 * (1 - 1e-12)


# --------------------------------------------------------------- features under noise
def test_prune_features_noisy_against_numpy_slicer(orc):
    """Noisy frames: the oracle's features against an independent numpy
    version (successive cancellation by explicit nearest-point search over
    the amplitudes, the distance to the decision boundaries by enumerating
    them).  A dropped outer clamp, a wrong spacing unit or a wrong sigma_r
    would each fail here."""
    for q, M, snr in ((4, 3, 4.0), (16, 4, 8.0), (64, 3, 14.0)):
        P = math.isqrt(q)
        f = gen_frames(M, M, q, snr, 40, seed=90 + q)
        R, z, _ = orc.qr(f.H, f.y)
        feat = orc.prune_features(R, z, P, f.sigma2)
        n = 2 * M
        c = math.sqrt(3.0 / (2.0 * (q - 1)))
        amps = (2 * np.arange(P) - (P - 1)) * c
        bounds = np.arange(-(P - 2), P - 1, 2) * c  # decision boundaries between neighbouring points
        sr = math.sqrt(f.sigma2 / 2)
        for b in range(len(f)):
            x = np.zeros(n)
            pd = 0.0
            for k in range(n - 1, -1, -1):
                ctr = z[b, k] - R[b, k, k + 1:] @ x[k + 1:]
                u = ctr / R[b, k, k]
                x[k] = amps[np.argmin(np.abs(amps - u))]
                pd += (ctr - R[b, k, k] * x[k]) ** 2
                d = np.min(np.abs(u - bounds)) / (2 * c)
                ref = [k / n, d, math.log2(R[b, k, k] * 2 * c / sr), pd / ((n - k) * sr * sr)]
                assert np.allclose(feat[b, k], ref, rtol=1e-9, atol=1e-12), (q, b, k)


# --------------------------------------------------------------- Adam over several steps
def test_adam_steps_closed_form(orc):
    """Steps t = 1..5 against Adam written out in closed form: m_t =
    (1 - b1) sum_i b1^(t-i) g_i, v_t = (1 - b2) sum_i b2^(t-i) g_i^2, with
    the bias corrections 1 - b^t; and a constant gradient, for which the
    corrected moments are g and g^2 exactly, so every step moves w by
    lr g / (|g| + eps)."""
    rng = np.random.default_rng(13)
    npar, lr, b1, b2, eps = 64, 3e-3, 0.9, 0.999, 1e-8
    gs = [rng.normal(size=npar) for _ in range(5)]
    w0 = rng.normal(size=npar)
    w, m, v = w0.copy(), np.zeros(npar), np.zeros(npar)
    wref = w0.copy()
    for t in range(1, 6):
        orc.adam_step(w, m, v, gs[t - 1], t, lr, b1, b2, eps)
        mt = (1 - b1) * sum(b1 ** (t - i) * gs[i - 1] for i in range(1, t + 1))
        vt = (1 - b2) * sum(b2 ** (t - i) * gs[i - 1] ** 2 for i in range(1, t + 1))
        wref = wref - lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(w, wref, rtol=1e-13, atol=1e-15), t
    g = rng.normal(size=npar)
    w, m, v = w0.copy(), np.zeros(npar), np.zeros(npar)
    for t in range(1, 6):
        orc.adam_step(w, m, v, g, t, lr, b1, b2, eps)
    assert np.allclose(w, w0 - 5 * lr * g / (np.abs(g) + eps), rtol=1e-10)


# --------------------------------------------------------------- the learned detector as a whole
def test_learned_detect_composition(orc):
    """The learned detector is the composition its definition states: with
    the noise test disabled its schedule is clamp(ceil(2^(f + margin))) of
    the MLP output on the SIC-path features (mapped here in numpy) and its
    result is K-best with that schedule; a huge margin gives the plain
    K-best with k_max survivors; a noise test that every frame fails gives
    the plain fallback K-best on every frame, flagged."""
    rng = np.random.default_rng(21)
    w = rng.normal(0, 0.2, orc.MLP_NPARAM)
    f = gen_frames(6, 6, 16, 12.0, 30, seed=95)
    R, z, _ = orc.qr(f.H, f.y)
    P, n, margin, kmin, kmax = 4, 12, 2.0, 1, 16
    out = orc.learned_detect(R, z, P, f.sigma2, w, margin, kmin, kmax, beta=1e9)
    feats = orc.prune_features(R, z, P, f.sigma2)
    pred = orc.mlp_forward(w, feats.reshape(-1, 4)).reshape(len(f), n)
    ks = np.clip(np.ceil(np.exp2(pred + margin)), kmin, kmax).astype(np.int32)
    assert np.array_equal(out["k_sched"], ks)
    assert len(np.unique(ks)) > 3
    kb = orc.kbest(R, z, P, kmax, k_sched=ks)
    assert np.array_equal(out["x"], kb["x"]) and np.allclose(out["pd"], kb["pd"], rtol=1e-14)
    assert not np.any(out["flags"] & orc.LEARNED_FALLBACK)
    big = orc.learned_detect(R, z, P, f.sigma2, w, 40.0, kmin, kmax, beta=1e9)
    assert np.all(big["k_sched"] == kmax) and np.array_equal(big["x"], orc.kbest(R, z, P, kmax)["x"])
    fb = orc.learned_detect(R, z, P, f.sigma2, w, margin, kmin, kmax, beta=-1e9, K_fallback=32)
    assert np.all(fb["flags"] & orc.LEARNED_FALLBACK)
    assert np.array_equal(fb["x"], orc.kbest(R, z, P, 32)["x"])

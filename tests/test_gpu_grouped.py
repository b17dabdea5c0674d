"""GPU parity of the grouped K-best (kbest_detect_grouped: J real levels per
step, the interference of the levels above each group of 16 from one
matrix-core product) with the FP64 oracle's K-best on the same tree
(orc.kbest with the same J).

The matrix product adds each R_kj a_j as three exact partial products, so
the FP32 pd bound is taken with three roundings per term (terms=3); the
mismatch rule is the forced-path near-tie rule of every K-best test."""
import math

import numpy as np
import pytest

from paper_2002_09561_amd.framegen import gen_frames
from tests.parity_util import check_kbest

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _case(gpu, orc, M, q, snr, B, K, J, seed, sched=None, radius=None):
    import torch

    f = gen_frames(M, M, q, snr, B, seed=seed)
    P = math.isqrt(q)
    print(f"grouped K-best J={J} {M}x{M} {q}-QAM {snr} dB B={B} K={K} seed={seed}", flush=True)
    H = torch.from_numpy(f.H).cuda()
    y = torch.from_numpy(f.y).cuda()
    R, z = gpu.qr_preprocess(H, y)
    ks = None if sched is None else torch.from_numpy(sched.astype(np.int32)).cuda()
    r2 = None if radius is None else torch.from_numpy(radius.astype(np.float32)).cuda()
    sym, pd, flags, ctr = gpu.kbest_detect_grouped(R, z, M, P, K, J=J, k_sched=ks, radius2=r2, want_counters=True)
    Ro, zo, _ = orc.qr(f.H, f.y)

    def ks_of(b):
        return None if sched is None else (sched if sched.ndim == 1 else sched[b:b + 1])

    def r2_of(b):
        return math.inf if radius is None else float(np.float32(radius[b]))

    if radius is None and (sched is None or sched.ndim == 1):
        out = orc.kbest(Ro, zo, P, K, k_sched=sched, J=J)
    else:
        parts = [orc.kbest(Ro[b:b + 1], zo[b:b + 1], P, K, k_sched=ks_of(b), r2=r2_of(b), J=J) for b in range(B)]
        out = {k: np.concatenate([p[k] for p in parts]) for k in ("x", "pd", "margin", "flags", "counters")}

    def forced(mask, xf):
        idx = np.nonzero(mask)[0]
        return np.array([orc.kbest(Ro[b:b + 1], zo[b:b + 1], P, K, J=J, force_path=xf[i:i + 1], k_sched=ks_of(b),
                                   r2=r2_of(b))["fgap"][0] for i, b in enumerate(idx)])

    return f, P, out, forced, Ro, zo, (_np(sym), _np(pd), _np(flags), _np(ctr))


def _check(orc, label, P, out, forced, Ro, zo, res):
    sym, pd, flags, ctr = res
    assert np.all((flags & 1) != 0) and np.all((out["flags"] & 1) != 0), label
    _, tol, nm = check_kbest(orc, label, P, orc.sym_to_x(sym, P), pd, out, Ro, zo, forced, terms=3)
    clean = out["margin"][:, 0] > tol  # no decision of the oracle within the near-tie window
    assert np.array_equal(ctr[clean, :2], out["counters"][clean, :2]), label
    return nm


@pytest.mark.parametrize("M,q,snr,B,K", [
    (4, 4, 10.0, 300, 16),     # one partial group (8 levels)
    (9, 16, 12.0, 150, 16),    # 18 levels: a full group under a group of 2
    (16, 16, 12.0, 150, 64),   # two full groups, 64 survivors (4 column tiles)
    (10, 64, 20.0, 100, 64),   # 64-QAM, 512 candidates per level
    (32, 16, 14.0, 60, 8),     # fewer than 16 survivors: one padded tile
    (64, 4, 6.0, 30, 32),
    (128, 4, 8.0, 4, 16),      # the largest size: 16 groups
    (7, 64, 16.0, 100, 1),     # K = 1: successive cancellation
    (100, 64, 24.0, 6, 64),    # plain K = 64 at 100x100 64-QAM
    (12, 64, 20.0, 80, 16),    # two blocks of children per lane (64-QAM, 9-16 survivors): the bound
    (20, 16, 14.0, 60, 32),    # two blocks (16-QAM, 17-32 survivors)
    (48, 4, 6.0, 30, 64),      # two blocks (4-QAM, 33-64 survivors)
])
def test_grouped_real_levels_parity(gpu, orc, M, q, snr, B, K):
    f, P, out, forced, Ro, zo, res = _case(gpu, orc, M, q, snr, B, K, 1, seed=9000 + 3 * M + K)
    nm = _check(orc, f"grouped J=1 {M}x{M} {q}-QAM K={K}", P, out, forced, Ro, zo, res)
    assert nm <= max(3, B // 20)
    n = 2 * M
    expect = sum(min(K, P ** t) for t in range(n))  # survivors expanded: closed form
    assert np.all(res[3][:, 0] == expect) and np.all(res[3][:, 1] == P * expect)


@pytest.mark.parametrize("M,q,snr,B,K", [
    (4, 16, 10.0, 200, 10),
    (8, 16, 12.0, 120, 64),    # 1024 candidates per step
    (16, 64, 18.0, 100, 10),
    (2, 4, 4.0, 100, 16),
    (24, 64, 22.0, 40, 16),
    (100, 64, 24.0, 6, 16),
])
def test_grouped_complex_levels_parity(gpu, orc, M, q, snr, B, K):
    f, P, out, forced, Ro, zo, res = _case(gpu, orc, M, q, snr, B, K, 2, seed=9500 + 3 * M + K)
    nm = _check(orc, f"grouped J=2 {M}x{M} {q}-QAM K={K}", P, out, forced, Ro, zo, res)
    assert nm <= max(3, B // 20)


def test_grouped_complex_node_count_is_papers(gpu, orc):
    """J = 2 at 16x16 64-QAM with K = 10: 1 + 15 K = 151 survivors expanded
    per frame, the visited-node count the paper prints."""
    f, P, out, forced, Ro, zo, res = _case(gpu, orc, 16, 64, 20.0, 40, 10, 2, seed=9600)
    assert np.all(res[3][:, 0] == 151) and np.all(res[3][:, 1] == 151 * 64 * 2)


def test_grouped_full_K_is_ml(gpu, orc):
    """2x2 4-QAM, J = 2 and K = 16 keeps every prefix: the exhaustive ML."""
    f, P, out, forced, Ro, zo, res = _case(gpu, orc, 2, 4, 3.0, 200, 16, 2, seed=9700)
    s_bf, _ = orc.brute_force(f.H, f.y, 4)
    assert np.allclose(orc.metric(f.H, f.y, res[0], 4), orc.metric(f.H, f.y, s_bf, 4), rtol=1e-9)


@pytest.mark.parametrize("J", [1, 2])
def test_grouped_schedule_and_radius(gpu, orc, J):
    """Per-frame schedules and radii around the ML metric: frames whose
    sphere holds no leaf are detected again without a radius (EMPTY_SPHERE
    with FOUND) on the GPU and in the oracle alike."""
    rng = np.random.default_rng(11 + J)
    M, q, B, K = 10, 16, 100, 16
    f0 = gen_frames(M, M, q, 9.0, B, seed=9800 + J)
    R0, z0, _ = orc.qr(f0.H, f0.y)
    ml = orc.sesd(R0, z0, 4)[1]
    radius = ml * rng.uniform(0.7, 2.0, B)
    sched = rng.integers(1, K + 1, (B, 2 * M)).astype(np.int32)
    f, P, out, forced, Ro, zo, res = _case(gpu, orc, M, q, 9.0, B, K, J, seed=9800 + J, sched=sched, radius=radius)
    flags = res[2]
    assert np.array_equal(flags & 3, out["flags"] & 3)
    assert np.any(flags & 2) and np.any(~flags & 2)
    _check(orc, f"grouped J={J} schedule+radius", P, out, forced, Ro, zo, res)


def test_grouped_nonfinite_frame(gpu, orc):
    """A NaN in R (in the top group's rows, or in a low row's entry of a
    level above its group) and an infinity in z stop their frames with
    NONFINITE_INPUT (sym 0, pd +inf); the other frames are detected as
    usual."""
    import torch

    from paper_2002_09561_amd import mimo

    M, q, B, K = 20, 16, 6, 16
    f = gen_frames(M, M, q, 12.0, B, seed=9900)
    R, z = gpu.qr_preprocess(torch.from_numpy(f.H).cuda(), torch.from_numpy(f.y).cuda())
    n = 2 * M
    R[1, 5] = float("nan")      # R[37][39]: a level of the top group
    R[4, (n - 1 - 3) * (n - 3) // 2 + (39 - 3)] = float("nan")  # R[3][39]: reaches level 3 through the matrix product
    z[3, 0] = float("inf")      # level 0 of frame 3
    for J in (1, 2):
        sym, pd, flags = gpu.kbest_detect_grouped(R, z, M, 4, K, J=J)
        fl, p, s = _np(flags), _np(pd), _np(sym)
        for b in (1, 3, 4):
            assert fl[b] & mimo.FLAG_NONFINITE_INPUT and not fl[b] & mimo.FLAG_FOUND
            assert np.isinf(p[b]) and np.all(s[b] == 0)
        for b in (0, 2, 5):
            assert fl[b] == mimo.FLAG_FOUND and np.isfinite(p[b])


def test_grouped_near_singular_channel(gpu, orc):
    """Columns 4 and 9 of H are made nearly parallel to their left
    neighbours (difference 0.05 times a Gaussian vector), so two diagonal
    entries of R are small and at their levels every survivor's children lie
    close together: most of the 512 candidates fall below the bound T.  (An
    FP64 simulation of this K-best puts more than 128 below T at 44% of the
    levels; at 29% more than 128 remain below the second bound as well.)  So
    both the second compaction and the sort of every block run here; the
    result must match the oracle under the near-tie rule, and the counters on
    frames without a near tie."""
    import torch

    M, q, B, K = 12, 64, 40, 64
    P = math.isqrt(q)
    f = gen_frames(M, M, q, 24.0, B, seed=9900)
    rng = np.random.default_rng(9901)
    H = f.H.copy()
    for c in (4, 9):
        d = (rng.standard_normal((B, M)) + 1j * rng.standard_normal((B, M))) / np.sqrt(2)
        H[:, :, c] = (H[:, :, c - 1] + 0.05 * d).astype(np.complex64)
    y = f.y
    print(f"grouped K-best near-singular {M}x{M} {q}-QAM B={B} K={K}", flush=True)
    R, z = gpu.qr_preprocess(torch.from_numpy(H).cuda(), torch.from_numpy(y).cuda())
    sym, pd, flags, ctr = gpu.kbest_detect_grouped(R, z, M, P, K, J=1, want_counters=True)
    Ro, zo, _ = orc.qr(H, y)
    out = orc.kbest(Ro, zo, P, K)

    def forced(mask, xf):
        return orc.kbest(Ro[mask], zo[mask], P, K, force_path=xf)["fgap"]

    res = (_np(sym), _np(pd), _np(flags), _np(ctr))
    _check(orc, f"grouped J=1 near-singular {M}x{M} {q}-QAM K={K}", P, out, forced, Ro, zo, res)
    expect = sum(min(K, P ** t) for t in range(2 * M))
    assert np.all(res[3][:, 0] == expect)

"""GPU parity of the complex-level K-best (pam^2 children per complex symbol,
the tree of the paper's figures) with the FP64 oracle's grouped K-best
(J = 2 real levels per step)."""
import math

import numpy as np
import pytest

from paper_2002_09561_amd.framegen import gen_frames
from tests.parity_util import check_kbest

pytestmark = pytest.mark.gpu


def _run(gpu, orc, M, q, snr, B, K, seed, sched=None, radius=None):
    import torch

    f = gen_frames(M, M, q, snr, B, seed=seed)
    P = math.isqrt(q)
    H = torch.from_numpy(f.H).cuda()
    y = torch.from_numpy(f.y).cuda()
    R, z = gpu.qr_preprocess(H, y)
    ks = None if sched is None else torch.from_numpy(sched.astype(np.int32)).cuda()
    r2 = None if radius is None else torch.from_numpy(radius.astype(np.float32)).cuda()
    print(f"complex K-best {M}x{M} {q}-QAM {snr} dB B={B} K={K}", flush=True)
    sym, pd, flags, ctr = gpu.kbest_detect_complex(R, z, M, P, K, k_sched=ks, radius2=r2, want_counters=True)
    Ro, zo, _ = orc.qr(f.H, f.y)
    if radius is None:
        out = orc.kbest(Ro, zo, P, K, k_sched=sched, J=2)
    else:
        parts = [orc.kbest(Ro[b:b + 1], zo[b:b + 1], P, K, k_sched=None if sched is None else sched[b:b + 1],
                           r2=float(np.float32(radius[b])), J=2) for b in range(B)]
        out = {k: np.concatenate([p[k] for p in parts]) for k in ("x", "pd", "margin", "flags", "counters")}
    Ro, zo, _ = orc.qr(f.H, f.y)

    def forced(mask, xf):
        idx = np.nonzero(mask)[0]
        return np.array([orc.kbest(Ro[b:b + 1], zo[b:b + 1], P, K, J=2, force_path=xf[i:i + 1],
                                   k_sched=None if sched is None else sched[b:b + 1],
                                   r2=math.inf if radius is None else float(np.float32(radius[b])))["fgap"][0]
                         for i, b in enumerate(idx)])
    out["forced"] = forced
    out["R"], out["z"] = Ro, zo
    return f, P, out, sym.cpu().numpy(), pd.cpu().numpy(), flags.cpu().numpy(), ctr.cpu().numpy()


def _check(orc, P, out, sym, pd, flags, ctr, label):
    """Symbols and search pd by the forced-path rule; counters on frames
    whose oracle run took no decision within the near-tie window."""
    assert np.all((flags & 1) != 0) and np.all((out["flags"] & 1) != 0), label
    _, tol, _ = check_kbest(orc, label, P, orc.sym_to_x(sym, P), pd, out, out["R"], out["z"], out["forced"])
    clean = out["margin"][:, 0] > tol
    assert np.array_equal(ctr[clean, :2], out["counters"][clean, :2]), label


def orc_sym(x, P):
    return (x[..., 0::2] * P + x[..., 1::2]).astype(np.int32)


@pytest.mark.parametrize("M,q,snr,B,K", [(4, 16, 10.0, 300, 10), (16, 16, 12.0, 200, 10), (16, 64, 18.0, 150, 10),
                                         (8, 64, 20.0, 100, 16), (32, 16, 14.0, 60, 64), (5, 4, 3.0, 100, 1),
                                         (6, 4, 2.0, 100, 24), (100, 64, 24.0, 6, 10), (12, 64, 20.0, 60, 32),
                                         (10, 64, 16.0, 60, 24)])
def test_kbest_complex_parity(gpu, orc, M, q, snr, B, K):
    f, P, out, sym, pd, flags, ctr = _run(gpu, orc, M, q, snr, B, K, seed=8000 + M * 7 + K)
    _check(orc, P, out, sym, pd, flags, ctr, f"complex K-best {M}x{M} {q}-QAM K={K}")


@pytest.mark.parametrize("K,nodes", [(10, 151), (32, 481)])
def test_kbest_complex_node_count_is_papers(gpu, orc, K, nodes):
    """Survivors expanded per frame = 1 + (M - 1) K for K <= |Omega|: at
    16x16 64-QAM, 151 for K = 10 and 481 for K = 32, the visited-node
    counts the paper prints (K = 32 has 2048 candidates per level)."""
    f, P, out, sym, pd, flags, ctr = _run(gpu, orc, 16, 64, 20.0, 50, K, seed=8100 + K)
    assert np.all(ctr[:, 0] == nodes)
    assert np.all(out["counters"][:, 0] == nodes)


def test_kbest_complex_full_K_is_ml(gpu, orc):
    """2x2 4-QAM with K = 16 keeps every prefix: the result is the exhaustive ML."""
    f, P, out, sym, pd, flags, ctr = _run(gpu, orc, 2, 4, 4.0, 200, 16, seed=8200)
    s_bf, _ = orc.brute_force(f.H, f.y, 4)
    m_gpu = orc.metric(f.H, f.y, sym, 4)
    m_bf = orc.metric(f.H, f.y, s_bf, 4)
    assert np.allclose(m_gpu, m_bf, rtol=1e-9)


def test_kbest_complex_schedule_and_radius(gpu, orc):
    rng = np.random.default_rng(5)
    M, q, B, K = 8, 16, 120, 16
    f0 = gen_frames(M, M, q, 9.0, B, seed=8300)
    R0, z0, _ = orc.qr(f0.H, f0.y)
    ml = orc.sesd(R0, z0, 4)[1]
    radius = ml * rng.uniform(0.7, 2.0, B)  # some spheres hold no K-best leaf
    sched = rng.integers(1, K + 1, (B, 2 * M)).astype(np.int32)
    f, P, out, sym, pd, flags, ctr = _run(gpu, orc, M, q, 9.0, B, K, seed=8300, sched=sched, radius=radius)
    # EMPTY_SPHERE (then detected again without a radius) on the same frames
    assert np.array_equal(flags & 3, out["flags"] & 3)
    assert np.any(flags & 2) and np.any(~flags & 2)
    _check(orc, P, out, sym, pd, flags, ctr, "complex K-best schedule+radius")

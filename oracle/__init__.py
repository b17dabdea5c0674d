"""FP64 CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import this package.  The product library never does,
and the two share no code: the oracle's arithmetic lives in ``oracle.c``
(plain C, FP64), this file only marshals numpy arrays into it.

See ``oracle.h`` for the conventions and the paper passage each routine
follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")

FOUND, EMPTY_SPHERE, BUDGET_EXHAUSTED, CERTIFIED, LEARNED_FALLBACK = 1, 2, 4, 8, 16
MLP_IN, MLP_H = 4, 128
MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_L = ctypes.c_int64


def _declare(L):
    L.orc_pam_scale.restype = _D
    L.orc_pam_scale.argtypes = [_I]
    L.orc_batch_qr.argtypes = [_I, _I, _I, _P, _P, _P, _P, _P]
    L.orc_batch_brute_force.argtypes = [_I, _I, _I, _I, _P, _P, _P, _P]
    L.orc_batch_metric.argtypes = [_I, _I, _I, _I, _P, _P, _P, _P]
    L.orc_batch_zf_sic.argtypes = [_I, _I, _I, _P, _P, _P, _P]
    L.orc_batch_qr_mmse.argtypes = [_I, _I, _I, _P, _P, _P, _P, _P]
    L.orc_batch_linear.argtypes = [_I, _I, _I, _P, _P, _P, _P]
    L.orc_batch_mrc.argtypes = [_I, _I, _I, _I, _P, _P, _P, _P]
    L.orc_batch_sesd.argtypes = [_I, _I, _I, _P, _P, _P, _L, _P, _P, _P, _P, _P]
    L.orc_batch_kbest.argtypes = [_I, _I, _I, _P, _P, _I, _P, _I, _D, _I, _P, _P, _P, _P, _P,
                                  _P, _P, _P, _P]
    L.orc_batch_hybrid.argtypes = [_I, _I, _I, _I, _P, _P, _P, _I, _I, _P, _I, _I, _L, _P, _P, _P,
                                   _P, _P]
    L.orc_batch_learned_detect.argtypes = [_I, _I, _I, _P, _P, _P, _P, _D, _I, _I, _D, _I, _P, _P, _P, _P]
    L.orc_hybrid_trace.restype = ctypes.c_uint32
    L.orc_hybrid_trace.argtypes = [_I, _I, _I, _P, _P, _D, _I, _I, _I, _L, _P, _P, _P, ctypes.c_char_p, _I]
    L.orc_batch_prune_features.argtypes = [_I, _I, _I, _P, _P, _P, _P]
    L.orc_path_terms.argtypes = [_I, _I, _P, _P, _P, _P]
    L.orc_mlp_forward.argtypes = [_P, _P, _I, _P]
    L.orc_mlp_loss_grad.restype = _D
    L.orc_mlp_loss_grad.argtypes = [_P, _P, _P, _I, _D, _P]
    L.orc_adam_step.argtypes = [_P, _P, _P, _P, _I, _I, _D, _D, _D, _D]


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def pam_scale(P: int) -> float:
    return lib().orc_pam_scale(P)


def amplitudes(P: int) -> np.ndarray:
    return (2.0 * np.arange(P) - (P - 1)) * pam_scale(P)


# ---------------------------------------------------------------- QR
def qr(H: np.ndarray, y: np.ndarray):
    """Sec. III-B.  H [B,N,M] complex64, y [B,N] complex64 ->
    R [B,n,n] (full, upper), z [B,n], resid [B] (all float64)."""
    H = _c(H, np.complex64)
    y = _c(y, np.complex64)
    B, N, M = H.shape
    n = 2 * M
    R = np.zeros((B, n, n))
    z = np.zeros((B, n))
    resid = np.zeros(B)
    lib().orc_batch_qr(B, N, M, _p(H), _p(y), _p(R), _p(z), _p(resid))
    return R, z, resid


def brute_force(H, y, qam: int):
    """Eq. (2): exhaustive ML -> (s_idx [B,M] int32, metric [B])."""
    H = _c(H, np.complex64)
    y = _c(y, np.complex64)
    B, N, M = H.shape
    P = math.isqrt(qam)
    s = np.zeros((B, M), np.int32)
    m = np.zeros(B)
    lib().orc_batch_brute_force(B, N, M, P, _p(H), _p(y), _p(s), _p(m))
    return s, m


def metric(H, y, s_idx, qam: int) -> np.ndarray:
    H = _c(H, np.complex64)
    y = _c(y, np.complex64)
    s_idx = _c(s_idx, np.int32)
    B, N, M = H.shape
    out = np.zeros(B)
    lib().orc_batch_metric(B, N, M, math.isqrt(qam), _p(H), _p(y), _p(s_idx), _p(out))
    return out


def zf_sic(R, z, P: int):
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    x = np.zeros((B, n), np.int32)
    pd = np.zeros(B)
    lib().orc_batch_zf_sic(B, n, P, _p(R), _p(z), _p(x), _p(pd))
    return x, pd


def qr_mmse(H, y, sigma2):
    """MMSE preprocessing: QR of [H; sigma I], [y; 0] in the real model.
    sigma2: scalar or [B] complex noise variances.  Returns R [B,n,n], z [B,n]
    with R^T R = H_r^T H_r + sigma2 I and R^T z = H_r^T y_r."""
    H = _c(H, np.complex64)
    y = _c(y, np.complex64)
    B, N, M = H.shape
    n = 2 * M
    s2 = _c(np.broadcast_to(np.asarray(sigma2, np.float64), (B,)), np.float64)
    R = np.zeros((B, n, n))
    z = np.zeros((B, n))
    lib().orc_batch_qr_mmse(B, N, M, _p(H), _p(y), _p(s2), _p(R), _p(z))
    return R, z


def linear(R, z, P: int):
    """Back-substitution without decision feedback (ZF on the plain QR,
    linear MMSE on the MMSE QR).  Returns (x_idx [B,n] int32, u [B,n])."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    x = np.zeros((B, n), np.int32)
    u = np.zeros((B, n))
    lib().orc_batch_linear(B, n, P, _p(R), _p(z), _p(x), _p(u))
    return x, u


def mrc(H, y, qam: int):
    """Maximum-ratio combining.  Returns (s_idx [B,M] int32, u [B,2M]) with u
    the interleaved (real, imaginary) estimates."""
    H = _c(H, np.complex64)
    y = _c(y, np.complex64)
    B, N, M = H.shape
    s = np.zeros((B, M), np.int32)
    u = np.zeros((B, 2 * M))
    lib().orc_batch_mrc(B, N, M, math.isqrt(qam), _p(H), _p(y), _p(s), _p(u))
    return s, u


def sesd(R, z, P: int, r2=None, budget: int = 0, x_init=None):
    """Alg. 1, Best-FS.  r2: None (= +inf) or [B] array.  Returns
    (x_idx [B,n], pd [B], flags [B], counters [B,4])."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    r2a = None if r2 is None else _c(np.broadcast_to(r2, (B,)), np.float64)
    xi = None if x_init is None else _c(x_init, np.int32)
    x = np.zeros((B, n), np.int32)
    pd = np.zeros(B)
    fl = np.zeros(B, np.uint32)
    ctr = np.zeros((B, 4), np.int64)
    lib().orc_batch_sesd(B, n, P, _p(R), _p(z), _p(r2a), int(budget), _p(xi), _p(x), _p(pd),
                         _p(fl), _p(ctr))
    return x, pd, fl, ctr


def kbest(R, z, P: int, K: int, k_sched=None, r2: float = math.inf, J: int = 1,
          force_path=None, want_rank: bool = False):
    """K-best (Sec. VI).  k_sched: None, [n] (shared) or [B,n] (per frame),
    indexed by level.  Returns dict with x, pd, margin [B,3], flags, counters
    and (if want_rank or force_path) rank [B,n]; with force_path also fgap [B],
    the largest relative gap of a decision that would have dropped the forced
    path (0 if it is the search's own result), and rgap [B,n], per step the
    smallest relative gap that could change the forced prefix's rank."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    ks, stride = None, 0
    if k_sched is not None:
        ks = _c(k_sched, np.int32)
        stride = n if ks.ndim == 2 else 0
    fp = None if force_path is None else _c(force_path, np.int32)
    x = np.zeros((B, n), np.int32)
    pd = np.zeros(B)
    mg = np.zeros((B, 3))
    rk = np.zeros((B, n), np.int32) if (want_rank or fp is not None) else None
    fg = np.zeros(B) if fp is not None else None
    rg = np.full((B, n), np.inf) if fp is not None else None
    fl = np.zeros(B, np.uint32)
    ctr = np.zeros((B, 4), np.int64)
    lib().orc_batch_kbest(B, n, P, _p(R), _p(z), int(K), _p(ks), stride, float(r2), int(J),
                          _p(fp), _p(x), _p(pd), _p(mg), _p(rk), _p(fg), _p(rg), _p(fl), _p(ctr))
    return dict(x=x, pd=pd, margin=mg, rank=rk, fgap=fg, rgap=rg, flags=fl, counters=ctr)


def hybrid(R, z, P: int, W: int, Kw: int, r2=math.inf, k_sched=None,
           master_off: bool = False, budget: int = 0, J: int = 1):
    """Hybrid SD-K-best in deterministic rounds (Sec. VI).  r2: scalar or [B];
    J real levels per step (2: one complex symbol, P^2 children)."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    r2a = _c(np.broadcast_to(np.asarray(r2, np.float64), (B,)), np.float64)
    ks, stride = None, 0
    if k_sched is not None:
        ks = _c(k_sched, np.int32)
        stride = n if ks.ndim == 2 else 0
    x = np.zeros((B, n), np.int32)
    pd = np.zeros(B)
    mg = np.zeros((B, 3))
    fl = np.zeros(B, np.uint32)
    ctr = np.zeros((B, 4), np.int64)
    lib().orc_batch_hybrid(B, n, P, int(J), _p(R), _p(z), _p(r2a), int(W), int(Kw), _p(ks), stride,
                           int(bool(master_off)), int(budget), _p(x), _p(pd), _p(mg), _p(fl),
                           _p(ctr))
    return dict(x=x, pd=pd, margin=mg, flags=fl, counters=ctr)


def hybrid_trace(R, z, P: int, W: int, Kw: int, r2: float = math.inf, master_off: bool = False,
                 budget: int = 0, J: int = 1):
    """One frame (R [n,n], z [n]) of the hybrid with its round-by-round text
    trace.  Returns (trace lines, x [n], pd, flags, counters [4])."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    n = z.shape[0]
    x = np.zeros(n, np.int32)
    pd = ctypes.c_double(0.0)
    ctr = np.zeros(4, np.int64)
    cap = 1 << 20
    buf = ctypes.create_string_buffer(cap)
    fl = lib().orc_hybrid_trace(n, P, int(J), _p(R), _p(z), float(r2), int(W), int(Kw), int(bool(master_off)),
                                int(budget), _p(x), ctypes.byref(pd), _p(ctr), buf, cap)
    return buf.value.decode().splitlines(), x, pd.value, int(fl), ctr


def path_terms(R, z, x, P: int) -> np.ndarray:
    """Eq. (4) terms g_k of one complete path (single frame)."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    x = _c(x, np.int32)
    n = z.shape[0]
    g = np.zeros(n)
    lib().orc_path_terms(n, P, _p(R), _p(z), _p(x), _p(g))
    return g


def prune_features(R, z, P: int, sigma2) -> np.ndarray:
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    s2 = _c(np.broadcast_to(sigma2, (B,)), np.float64)
    f = np.zeros((B, n, 4))
    lib().orc_batch_prune_features(B, n, P, _p(R), _p(z), _p(s2), _p(f))
    return f


def learned_detect(R, z, P: int, sigma2, w, margin: float, k_min: int, k_max: int, beta: float,
                   K_fallback: int = 64):
    """The learned-pruning detector (features -> MLP -> survivor schedule ->
    K-best -> plain K-best fallback), FP64.  sigma2 scalar or [B].  Returns
    dict with x [B,n], pd [B], k_sched [B,n], flags [B]."""
    R = _c(R, np.float64)
    z = _c(z, np.float64)
    B, n = z.shape
    s2 = _c(np.broadcast_to(np.asarray(sigma2, np.float64), (B,)), np.float64)
    w = _c(w, np.float64)
    x = np.zeros((B, n), np.int32)
    pd = np.zeros(B)
    ks = np.zeros((B, n), np.int32)
    fl = np.zeros(B, np.uint32)
    lib().orc_batch_learned_detect(B, n, P, _p(R), _p(z), _p(s2), _p(w), float(margin), int(k_min), int(k_max),
                                   float(beta), int(K_fallback), _p(x), _p(pd), _p(ks), _p(fl))
    return dict(x=x, pd=pd, k_sched=ks, flags=fl)


# ---------------------------------------------------------------- MLP
def mlp_forward(w, X) -> np.ndarray:
    w = _c(w, np.float64)
    X = _c(X, np.float64)
    out = np.zeros(X.shape[0])
    lib().orc_mlp_forward(_p(w), _p(X), X.shape[0], _p(out))
    return out


def mlp_loss_grad(w, X, y, tau: float = 0.95):
    w = _c(w, np.float64)
    X = _c(X, np.float64)
    y = _c(y, np.float64)
    g = np.zeros(MLP_NPARAM)
    loss = lib().orc_mlp_loss_grad(_p(w), _p(X), _p(y), X.shape[0], float(tau), _p(g))
    return loss, g


def adam_step(w, m, v, g, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays w, m, v."""
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _c(g, np.float64)
    lib().orc_adam_step(_p(w), _p(m), _p(v), _p(g), w.size, int(t), float(lr), float(beta1),
                        float(beta2), float(eps))


# ---------------------------------------------------------------- conversions
def x_to_sym(x: np.ndarray, P: int) -> np.ndarray:
    """Real-level PAM indices [.., 2M] -> QAM indices [.., M] (i_re * P + i_im)."""
    return (x[..., 0::2] * P + x[..., 1::2]).astype(np.int32)


def sym_to_x(s: np.ndarray, P: int) -> np.ndarray:
    x = np.empty(s.shape[:-1] + (2 * s.shape[-1],), np.int32)
    x[..., 0::2] = s // P
    x[..., 1::2] = s % P
    return x


def gray_bits(s_idx: np.ndarray, P: int) -> np.ndarray:
    """Gray-coded bits of QAM indices: Gray(i_re) || Gray(i_im), MSB first."""
    b = int(round(math.log2(P)))
    ire, iim = s_idx // P, s_idx % P
    gre, gim = ire ^ (ire >> 1), iim ^ (iim >> 1)
    code = (gre << b) | gim
    shifts = np.arange(2 * b - 1, -1, -1)
    return ((code[..., None] >> shifts) & 1).astype(np.uint8)


def error_counts(s_hat: np.ndarray, s_ref: np.ndarray, P: int):
    """(bit errors, symbol errors) between two QAM-index arrays."""
    bits = (gray_bits(s_hat, P) != gray_bits(s_ref, P)).sum()
    syms = (s_hat != s_ref).sum()
    return int(bits), int(syms)

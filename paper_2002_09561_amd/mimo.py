"""Python binding of the C ABI in include/mimo_sd.h (libmimo_sd.so).

Argument marshalling only: every step of the detection path runs in the HIP
kernels of the library.  Tensors must be CUDA (HIP) tensors on the current
device, contiguous and of the dtype stated; outputs are allocated here with
torch and filled by the library on torch's current stream.  There is no CPU
fallback: if the library is not built, or the GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmimo_sd.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP = 0, -1, -2, -3, -4
FLAG_FOUND, FLAG_EMPTY_SPHERE, FLAG_BUDGET_EXHAUSTED, FLAG_CERTIFIED, FLAG_LEARNED_FALLBACK = 1, 2, 4, 8, 16
FLAG_NONFINITE_INPUT, FLAG_INVALID_FRAME = 32, 64
MLP_IN, MLP_HIDDEN = 4, 128
MLP_NPARAM = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
MAX_WORKERS = 15

# exported symbols and their C signatures (argument types, return type)
_P, _I32, _I64, _F, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
SIGNATURES = {
    "mimo_last_error": ([], ctypes.c_char_p),
    "mimo_version": ([], _I32),
    "mimo_qr_preprocess": ([_P, _P, _I32, _I32, _I32, _P, _P, _P, _P], _I32),
    "mimo_qr_preprocess_mmse": ([_P, _P, _P, _I32, _I32, _I32, _P, _P, _P], _I32),
    "linear_detect": ([_P, _P, _I32, _I32, _I32, _P, _P, _P], _I32),
    "mrc_detect": ([_P, _P, _I32, _I32, _I32, _I32, _P, _P, _P], _I32),
    "mimo_paper_radius2": ([_P, _I32, _I32, _I32, _P, _P], _I32),
    "kbest_detect": ([_P, _P, _I32, _I32, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _P], _I32),
    "kbest_detect_complex": ([_P, _P, _I32, _I32, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _P], _I32),
    "kbest_detect_grouped": ([_P, _P, _I32, _I32, _I32, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P, _P], _I32),
    "kbest_fallback_mark": ([_P, _P, _P, _I32, _I32, _F, _P], _I32),
    "mimo_metric_select": ([_P, _P, _P, _P, ctypes.c_uint32, ctypes.c_uint32, _I32, _I32, _I32, _I32, _P, _P], _I32),
    "kbest_rank_labels": ([_P, _P, _I32, _I32, _I32, _I32, _P, _P, _P], _I32),
    "kbest_fallback": ([_P, _P, _I32, _I32, _I32, _I32, _P, _F, _P, _P, _P, _P, _P], _I32),
    "sd_hybrid_detect": ([_P, _P, _I32, _I32, _I32, _P, _I32, _I32, _P, _I32, _I32, _I64, _P, _P, _P, _P,
                          _P], _I32),
    "sd_hybrid_detect_complex": ([_P, _P, _I32, _I32, _I32, _P, _I32, _I32, _P, _I32, _I32, _I64, _P, _P, _P, _P,
                          _P], _I32),
    "sd_parallel_detect": ([_P, _P, _I32, _I32, _I32, _P, _I64, _I32, _P, _P, _P, _P, _P], _I32),
    "mimo_metric": ([_P, _P, _P, _I32, _I32, _I32, _I32, _P, _P], _I32),
    "mimo_error_count": ([_P, _P, _I32, _I32, _I32, _P, _P], _I32),
    "prune_features": ([_P, _P, _P, _I32, _I32, _I32, _P, _P], _I32),
    "prune_mlp_forward": ([_P, _P, _I64, _P, _P], _I32),
    "prune_mlp_schedule": ([_P, _P, _I64, _F, _I32, _I32, _I32, _P, _P, _P], _I32),
    "prune_mlp_workspace_bytes": ([_I64], _SZ),
    "prune_mlp_loss_grad": ([_P, _P, _P, _I64, _F, _P, _P, _P, _SZ, _P], _I32),
    "prune_mlp_loss_grad_noalloc": ([_P, _P, _P, _I64, _F, _P, _P, _P], _I32),
    "prune_mlp_adam_step": ([_P, _P, _P, _P, _I32, _I32, _F, _F, _F, _F, _P], _I32),
    "mimo_qr_preprocess_uneven": ([_P, _I32, _I32, _P, _P, _P, _P, _P, _I32, _P], _I32),
    "kbest_detect_uneven": ([_P, _I32, _P, _P, _P, _P, _P, _P, _I32, _P], _I32),
}


class MimoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def load(path: str | None = None):
    """Load libmimo_sd.so (built by paper_2002_09561_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built; run paper_2002_09561_amd.build.build() first")
    lib = ctypes.CDLL(p)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        raise MimoError(rc, load().mimo_last_error().decode())


def _ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def packed_size(n: int) -> int:
    return n * (n + 1) // 2


# ------------------------------------------------------------------ QR
def qr_preprocess(H: torch.Tensor, y: torch.Tensor, want_resid: bool = False, out=None, stream=None):
    """H [B,N,M] complex64, y [B,N] complex64 -> R [B, n(n+1)/2], z [B, n] (and resid [B])."""
    B, N, M = H.shape
    n = 2 * M
    dev = H.device
    if out is None:
        R = torch.empty(B, packed_size(n), device=dev, dtype=torch.float32)
        z = torch.empty(B, n, device=dev, dtype=torch.float32)
        resid = torch.empty(B, device=dev, dtype=torch.float32) if want_resid else None
    else:
        R, z, resid = out
    _check(load().mimo_qr_preprocess(_ptr(H, torch.complex64, "H"), _ptr(y, torch.complex64, "y"), B, N, M,
                                     _ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"),
                                     _ptr(resid, torch.float32, "resid"), _stream(stream)))
    return (R, z, resid) if want_resid else (R, z)


def qr_preprocess_mmse(H: torch.Tensor, y: torch.Tensor, sigma2: torch.Tensor, out=None, stream=None):
    """QR of [H; sigma I], [y; 0] (MMSE preprocessing).  sigma2 [B] float32.
    Returns R [B, n(n+1)/2], z [B, n] as qr_preprocess."""
    B, N, M = H.shape
    n = 2 * M
    if out is None:
        R = torch.empty(B, packed_size(n), device=H.device, dtype=torch.float32)
        z = torch.empty(B, n, device=H.device, dtype=torch.float32)
    else:
        R, z = out
    _check(load().mimo_qr_preprocess_mmse(_ptr(H, torch.complex64, "H"), _ptr(y, torch.complex64, "y"),
                                          _ptr(sigma2, torch.float32, "sigma2"), B, N, M,
                                          _ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), _stream(stream)))
    return R, z


def paper_radius2(n_rx: int, n_tx: int, sigma2: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """The paper's sphere radius rule, squared: r^2 = N M sigma^2 per frame
    (mimo_paper_radius2).  sigma2 [B] float32 on the device."""
    B = sigma2.shape[0]
    r2 = out if out is not None else torch.empty(B, device=sigma2.device, dtype=torch.float32)
    _check(load().mimo_paper_radius2(_ptr(sigma2, torch.float32, "sigma2"), B, n_rx, n_tx,
                                     _ptr(r2, torch.float32, "radius2"), _stream(stream)))
    return r2


# ------------------------------------------------------------------ detectors
def linear_detect(R, z, n_tx: int, pam: int, want_xhat: bool = False, stream=None):
    """Back-substitution without decision feedback (ZF on the plain QR, linear
    MMSE on the MMSE QR).  Returns sym [B, n_tx] int32 (and xhat [B, n])."""
    B = z.shape[0]
    sym = torch.empty(B, n_tx, device=z.device, dtype=torch.int32)
    xh = torch.empty(B, 2 * n_tx, device=z.device, dtype=torch.float32) if want_xhat else None
    _check(load().linear_detect(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam, _ptr(sym),
                                _ptr(xh), _stream(stream)))
    return (sym, xh) if want_xhat else sym


def mrc_detect(H, y, pam: int, want_xhat: bool = False, stream=None):
    """Maximum-ratio combining.  Returns sym [B, M] int32 (and xhat [B, 2M])."""
    B, N, M = H.shape
    sym = torch.empty(B, M, device=H.device, dtype=torch.int32)
    xh = torch.empty(B, 2 * M, device=H.device, dtype=torch.float32) if want_xhat else None
    _check(load().mrc_detect(_ptr(H, torch.complex64, "H"), _ptr(y, torch.complex64, "y"), B, N, M, pam, _ptr(sym),
                             _ptr(xh), _stream(stream)))
    return (sym, xh) if want_xhat else sym


def _det_outputs(B, n_tx, dev, want_counters):
    sym = torch.empty(B, n_tx, device=dev, dtype=torch.int32)
    pd = torch.empty(B, device=dev, dtype=torch.float32)
    flags = torch.empty(B, device=dev, dtype=torch.int32)
    ctr = torch.empty(B, 4, device=dev, dtype=torch.int64) if want_counters else None
    return sym, pd, flags, ctr


def _sched(k_sched, n):
    if k_sched is None:
        return None, 0
    if k_sched.dim() == 1:
        return k_sched, 0
    return k_sched, n


def kbest_detect(R, z, n_tx: int, pam: int, K: int, k_sched=None, radius2=None, want_counters=False,
                 out=None, stream=None):
    """Batched K-best.  Returns (sym [B,n_tx] int32, pd [B] f32, flags [B] int32[, counters])."""
    B = z.shape[0]
    n = 2 * n_tx
    sym, pd, flags, ctr = out if out is not None else _det_outputs(B, n_tx, z.device, want_counters)
    ks, stride = _sched(k_sched, n)
    _check(load().kbest_detect(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam, K,
                               _ptr(ks, torch.int32, "k_sched"), stride, _ptr(radius2, torch.float32, "radius2"),
                               _ptr(sym), _ptr(pd), _ptr(flags), _ptr(ctr), _stream(stream)))
    return (sym, pd, flags, ctr) if want_counters else (sym, pd, flags)


def kbest_detect_complex(R, z, n_tx: int, pam: int, K: int, k_sched=None, radius2=None, want_counters=False,
                         out=None, stream=None):
    """Batched K-best over complex levels (pam^2 children per level).
    Returns (sym [B,n_tx] int32, pd [B] f32, flags [B] int32[, counters])."""
    B = z.shape[0]
    n = 2 * n_tx
    sym, pd, flags, ctr = out if out is not None else _det_outputs(B, n_tx, z.device, want_counters)
    ks, stride = _sched(k_sched, n)
    _check(load().kbest_detect_complex(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam, K,
                                       _ptr(ks, torch.int32, "k_sched"), stride,
                                       _ptr(radius2, torch.float32, "radius2"), _ptr(sym), _ptr(pd), _ptr(flags),
                                       _ptr(ctr), _stream(stream)))
    return (sym, pd, flags, ctr) if want_counters else (sym, pd, flags)


def kbest_detect_grouped(R, z, n_tx: int, pam: int, K: int, J: int = 1, k_sched=None, radius2=None,
                         want_counters=False, out=None, stream=None):
    """Grouped K-best (J real levels per step; the interference of the levels
    above each group of 16 from one matrix product).  Same tree and outputs
    as kbest_detect (J = 1) or kbest_detect_complex (J = 2).
    Returns (sym [B,n_tx] int32, pd [B] f32, flags [B] int32[, counters])."""
    B = z.shape[0]
    n = 2 * n_tx
    sym, pd, flags, ctr = out if out is not None else _det_outputs(B, n_tx, z.device, want_counters)
    ks, stride = _sched(k_sched, n)
    _check(load().kbest_detect_grouped(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam, K, J,
                                       _ptr(ks, torch.int32, "k_sched"), stride,
                                       _ptr(radius2, torch.float32, "radius2"), _ptr(sym), _ptr(pd), _ptr(flags),
                                       _ptr(ctr), _stream(stream)))
    return (sym, pd, flags, ctr) if want_counters else (sym, pd, flags)


def kbest_fallback(R, z, n_tx: int, pam: int, K: int, sigma2, beta: float, out, counters=None, stream=None):
    """Re-detect with plain K-best the frames of `out` = (sym, pd, flags) whose
    learned detection is flagged or whose metric exceeds the noise bound."""
    B = z.shape[0]
    sym, pd, flags = out[:3]
    _check(load().kbest_fallback(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam, K,
                                 _ptr(sigma2, torch.float32, "sigma2"), float(beta), _ptr(sym, torch.int32, "sym"),
                                 _ptr(pd, torch.float32, "pd"), _ptr(flags, torch.int32, "flags"),
                                 _ptr(counters, torch.int64, "counters"), _stream(stream)))
    return sym, pd, flags


def kbest_fallback_mark(n_tx: int, sigma2, beta: float, out, stream=None):
    """Flag (FLAG_LEARNED_FALLBACK) the frames of `out` = (sym, pd, flags) that
    kbest_fallback would detect again."""
    pd, flags = out[1], out[2]
    B = pd.shape[0]
    _check(load().kbest_fallback_mark(_ptr(pd, torch.float32, "pd"), _ptr(flags, torch.int32, "flags"),
                                      _ptr(sigma2, torch.float32, "sigma2"), B, n_tx, float(beta), _stream(stream)))
    return flags


def kbest_rank_labels(R, z, n_tx: int, pam: int, K: int, force_sym, stream=None):
    B = z.shape[0]
    rank = torch.empty(B, 2 * n_tx, device=z.device, dtype=torch.int32)
    _check(load().kbest_rank_labels(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam, K,
                                    _ptr(force_sym, torch.int32, "force_sym"), _ptr(rank), _stream(stream)))
    return rank


def sd_hybrid_detect(R, z, n_tx: int, pam: int, n_workers: int, k_worker: int, radius2=None, k_sched=None,
                     master_off=False, node_budget: int = 0, want_counters=False, out=None, stream=None,
                     complex_levels=False):
    """Hybrid SD / K-best.  complex_levels=True runs sd_hybrid_detect_complex:
    one complex symbol (pam^2 children) per tree step."""
    B = z.shape[0]
    n = 2 * n_tx
    sym, pd, flags, ctr = out if out is not None else _det_outputs(B, n_tx, z.device, want_counters)
    ks, stride = _sched(k_sched, n)
    fn = load().sd_hybrid_detect_complex if complex_levels else load().sd_hybrid_detect
    _check(fn(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam,
              _ptr(radius2, torch.float32, "radius2"), n_workers, k_worker,
              _ptr(ks, torch.int32, "k_sched"), stride, int(bool(master_off)),
              int(node_budget), _ptr(sym), _ptr(pd), _ptr(flags), _ptr(ctr),
              _stream(stream)))
    return (sym, pd, flags, ctr) if want_counters else (sym, pd, flags)


def sd_parallel_detect(R, z, n_tx: int, pam: int, radius2=None, node_budget: int = 0, redo: bool = False,
                       want_counters=False, out=None, stream=None):
    """Exact SD with each frame's tree spread over the wavefronts of one
    workgroup.  redo=True: only frames of `out` = (sym, pd, flags[, counters])
    left unfinished (BUDGET_EXHAUSTED, no CERTIFIED) by an earlier search are
    searched again, in place.  Returns (sym, pd, flags[, counters])."""
    B = z.shape[0]
    if redo and out is None:
        raise ValueError("redo needs the earlier search's outputs in `out`")
    if out is not None:
        sym, pd, flags = out[:3]
        ctr = out[3] if len(out) > 3 else None
    else:
        sym, pd, flags, ctr = _det_outputs(B, n_tx, z.device, want_counters)
    _check(load().sd_parallel_detect(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"), B, n_tx, pam,
                                     _ptr(radius2, torch.float32, "radius2"), int(node_budget), int(bool(redo)),
                                     _ptr(sym), _ptr(pd), _ptr(flags), _ptr(ctr), _stream(stream)))
    return (sym, pd, flags, ctr) if want_counters else (sym, pd, flags)


# ------------------------------------------------------------------ epilogues
def metric(H, y, sym, pam: int, out=None, stream=None):
    B, N, M = H.shape
    m = out if out is not None else torch.empty(B, device=H.device, dtype=torch.float64)
    _check(load().mimo_metric(_ptr(H, torch.complex64, "H"), _ptr(y, torch.complex64, "y"),
                              _ptr(sym, torch.int32, "sym"), B, N, M, pam, _ptr(m, torch.float64), _stream(stream)))
    return m


def metric_select(H, y, sym, pam: int, flags, mask: int, value: int, out, stream=None):
    """FP64 metric of the frames with (flags & mask) == value, into `out`."""
    B, N, M = H.shape
    _check(load().mimo_metric_select(_ptr(H, torch.complex64, "H"), _ptr(y, torch.complex64, "y"),
                                     _ptr(sym, torch.int32, "sym"), _ptr(flags, torch.int32, "flags"), int(mask),
                                     int(value), B, N, M, pam, _ptr(out, torch.float64), _stream(stream)))
    return out


def error_count(sym, ref, pam: int, counts=None, stream=None):
    """counts (int64 [3], accumulated): bit errors, symbol errors, frames in error."""
    B, M = sym.shape
    c = counts if counts is not None else torch.zeros(3, device=sym.device, dtype=torch.int64)
    _check(load().mimo_error_count(_ptr(sym, torch.int32, "sym"), _ptr(ref, torch.int32, "ref"), B, M, pam,
                                   _ptr(c, torch.int64, "counts"), _stream(stream)))
    return c


def prune_features(R, z, sigma2, n_tx: int, pam: int, out=None, stream=None):
    B = z.shape[0]
    f = out if out is not None else torch.empty(B, 2 * n_tx, 4, device=z.device, dtype=torch.float32)
    _check(load().prune_features(_ptr(R, torch.float32, "R"), _ptr(z, torch.float32, "z"),
                                 _ptr(sigma2, torch.float32, "sigma2"), B, n_tx, pam, _ptr(f), _stream(stream)))
    return f


# ------------------------------------------------------------------ MLP
def mlp_forward(w, X, out=None, stream=None):
    S = X.shape[0]
    o = out if out is not None else torch.empty(S, device=X.device, dtype=torch.float32)
    _check(load().prune_mlp_forward(_ptr(w, torch.float32, "w"), _ptr(X, torch.float32, "X"), S, _ptr(o),
                                    _stream(stream)))
    return o


def mlp_schedule(w, X, n: int, margin: float, k_min: int, k_max: int, flags=None, out=None, stream=None):
    S = X.shape[0]
    ks = out if out is not None else torch.empty(S, device=X.device, dtype=torch.int32)
    _check(load().prune_mlp_schedule(_ptr(w, torch.float32, "w"), _ptr(X, torch.float32, "X"), S, float(margin),
                                     int(k_min), int(k_max), int(n), _ptr(ks), _ptr(flags, torch.int32, "flags"),
                                     _stream(stream)))
    return ks


def mlp_workspace_bytes(S: int) -> int:
    return int(load().prune_mlp_workspace_bytes(S))


def mlp_loss_grad(w, X, y, tau: float, ws=None, grad=None, loss=None, stream=None):
    S = X.shape[0]
    nb = mlp_workspace_bytes(S)
    if ws is None:
        ws = torch.empty(nb, device=X.device, dtype=torch.uint8)
    g = grad if grad is not None else torch.empty(w.numel(), device=X.device, dtype=torch.float32)
    l = loss if loss is not None else torch.empty(1, device=X.device, dtype=torch.float32)
    _check(load().prune_mlp_loss_grad(_ptr(w, torch.float32, "w"), _ptr(X, torch.float32, "X"),
                                      _ptr(y, torch.float32, "y"), S, float(tau), _ptr(g), _ptr(l), _ptr(ws),
                                      ws.numel() * ws.element_size(), _stream(stream)))
    return l, g


MLP_NOALLOC_MAX_S = 8192


def mlp_loss_grad_noalloc(w, X, y, tau: float, grad, loss, stream=None):
    """prune_mlp_loss_grad without a workspace (the library's static scratch,
    S <= MLP_NOALLOC_MAX_S); grad [NPARAM] and loss [1] float32 are given by
    the caller, so this call allocates nothing."""
    S = X.shape[0]
    _check(load().prune_mlp_loss_grad_noalloc(_ptr(w, torch.float32, "w"), _ptr(X, torch.float32, "X"),
                                              _ptr(y, torch.float32, "y"), S, float(tau),
                                              _ptr(grad, torch.float32, "grad"), _ptr(loss, torch.float32, "loss"),
                                              _stream(stream)))
    return loss, grad


def mlp_adam_step(w, m, v, g, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(load().prune_mlp_adam_step(_ptr(w, torch.float32, "w"), _ptr(m, torch.float32, "m"),
                                      _ptr(v, torch.float32, "v"), _ptr(g, torch.float32, "g"), w.numel(), int(t),
                                      float(lr), float(beta1), float(beta2), float(eps), _stream(stream)))


# ------------------------------------------------------------------ uneven batches
def qr_preprocess_uneven(desc, B: int, max_rx: int, H_flat, y_flat, R_flat, z_flat, counter, grid: int = 0,
                         stream=None):
    """desc: uint8 tensor holding B mimo_frame_desc records (56 bytes each)."""
    _check(load().mimo_qr_preprocess_uneven(_ptr(desc, torch.uint8, "desc"), B, max_rx,
                                            _ptr(H_flat, torch.complex64, "H_flat"),
                                            _ptr(y_flat, torch.complex64, "y_flat"), _ptr(R_flat, torch.float32, "R"),
                                            _ptr(z_flat, torch.float32, "z"), _ptr(counter, torch.int32, "counter"),
                                            int(grid), _stream(stream)))


def kbest_detect_uneven(desc, B: int, R_flat, z_flat, sym_flat, pd, flags, counter, grid: int = 0, stream=None):
    _check(load().kbest_detect_uneven(_ptr(desc, torch.uint8, "desc"), B, _ptr(R_flat, torch.float32, "R"),
                                      _ptr(z_flat, torch.float32, "z"), _ptr(sym_flat, torch.int32, "sym"),
                                      _ptr(pd, torch.float32, "pd"), _ptr(flags, torch.int32, "flags"),
                                      _ptr(counter, torch.int32, "counter"), int(grid), _stream(stream)))

"""Helpers shared by the GPU parity tests (test-side code only)."""
import math

import numpy as np

# Near-tie window for FP32 detections against the FP64 oracle.  A symbol
# mismatch is excused iff one of the oracle's own decisions on that frame
# (a selection boundary, a radius test or the final choice) compared two
# values whose relative gap is at most NEAR_TIE.  The FP32 partial distances
# carry a relative error of a few 1e-6 at 16x16 and up to ~2e-5 at 100x100
# (FP32 QR and FP32 accumulation; measured in the parity tests), so the
# window is 1e-5 for n <= 64 and 5e-5 beyond.
def near_tie_tol(n: int) -> float:
    return 1e-5 if n <= 64 else 5e-5


def pack_level_order(R: np.ndarray) -> np.ndarray:
    """Full upper-triangular [B, n, n] -> packed level order [B, n(n+1)/2]."""
    B, n, _ = R.shape
    out = np.empty((B, n * (n + 1) // 2), R.dtype)
    off = 0
    for k in range(n - 1, -1, -1):
        out[:, off: off + n - k] = R[:, k, k:]
        off += n - k
    return out


def compare_symbols(sym_gpu, sym_orc, margin, tol, label=""):
    """Returns (n_mismatch, n_excused); asserts every mismatch is a near tie."""
    sym_gpu = np.asarray(sym_gpu)
    mism = np.any(sym_gpu != sym_orc, axis=1)
    excused = mism & (margin[:, 0] <= tol)
    bad = np.nonzero(mism & ~excused)[0]
    if bad.size:
        lines = [f"{label}: {bad.size} unexcused mismatches of {len(mism)} frames"]
        for b in bad[:5]:
            lines.append(f"  frame {b}: oracle margin {margin[b, 0]:.3e} ({margin[b, 1]:.6g} vs {margin[b, 2]:.6g})")
        raise AssertionError("\n".join(lines))
    if mism.any():
        print(f"{label}: {mism.sum()} near-tie mismatches excused (margins "
              f"{np.array2string(margin[mism, 0][:5], precision=2)})")
    return int(mism.sum()), int(excused.sum())


def qam_P(qam: int) -> int:
    return math.isqrt(qam)

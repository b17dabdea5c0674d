"""Helpers shared by the GPU parity tests (test-side code only).

How a GPU detection is compared with the FP64 oracle on the same frames:

* The GPU searches in FP32 on R and z rounded to FP32; the oracle in FP64.
  Where both return the same path, the GPU's search pd must lie within
  `pd_error_bound` of the oracle's pd of that path (a first-order bound
  derived from the FP32 arithmetic, not fitted).  The largest relative error
  seen on the matched frames is the configuration's measured eps_FP32; it is
  logged with every comparison.
* Where the paths differ, the oracle is run again with the GPU's path forced
  to survive (`orc.kbest(..., force_path=...)`).  The mismatch is excused iff
  every decision that would have dropped that path, or preferred another
  leaf, compared two keys within the near-tie window
  tol = max(1e-5, 2 eps_FP32) of each other (each of the two keys carries up
  to eps_FP32 of rounding, so such a pair can come out in either order).
  Nothing else excuses a mismatch.
"""
import math

import numpy as np

U32 = 2.0 ** -24
NEAR_TIE_FLOOR = 1e-5


def near_tie_tol(eps_fp32: float) -> float:
    """Near-tie window from the measured FP32 error of the search pd."""
    return max(NEAR_TIE_FLOOR, 2.0 * eps_fp32)


def pam_scale(P: int) -> float:
    return math.sqrt(3.0 / (2.0 * (P * P - 1)))


def pack_level_order(R: np.ndarray) -> np.ndarray:
    """Full upper-triangular [B, n, n] -> packed level order [B, n(n+1)/2]."""
    B, n, _ = R.shape
    out = np.empty((B, n * (n + 1) // 2), R.dtype)
    off = 0
    for k in range(n - 1, -1, -1):
        out[:, off: off + n - k] = R[:, k, k:]
        off += n - k
    return out


def pd_error_bound(R, z, x, P, terms=3):
    """Per-frame bound on |pd_FP32 - pd_FP64| of the path x [B, n] (PAM
    indices) for a search that holds R and z rounded to FP32 (relative 2^-24
    per entry), scales R by the PAM spacing in FP32 (one more rounding), sums
    the centre b_k = z_k - sum_{j>k} R_kj a_j with FP32 additions in any
    order (gamma, terms * m roundings for m terms: terms = 3 when every
    R_kj a_j enters as three exact partial products, as on the matrix cores
    with c R split into three bf16 parts), forms e_k = b_k - R_kk a_k and
    pd += e_k^2 with one rounding each.  First order in u = 2^-24;
    second-order terms are covered by the factor 1.5.  The default terms = 3
    covers both centre forms the K-best entry points use (one FMA per term,
    or three exact partial products per term on the matrix cores)."""
    R = np.asarray(R, np.float64)
    z = np.asarray(z, np.float64)
    B, n = z.shape
    amp = (2.0 * np.asarray(x, np.float64) - (P - 1)) * pam_scale(P)
    T = np.abs(np.triu(R, 1) * amp[:, None, :])             # |R_kj a_j|, j > k
    S = np.abs(z) + T.sum(axis=2)                             # per level
    m = np.arange(n)[None, :]                                  # terms above level k ...
    m = (n - 1 - m).astype(np.float64)                         # ... n - 1 - k of them
    db = (terms * m + 4.0) * U32 * S
    diag = np.abs(np.einsum("bkk->bk", R) * amp)
    e = z - (np.triu(R) * amp[:, None, :]).sum(axis=2)
    de = db + 2.0 * U32 * diag + U32 * np.abs(e)
    pd = (e * e).sum(axis=1)
    return 1.5 * ((2.0 * np.abs(e) * de + de * de).sum(axis=1) + n * U32 * pd)


def check_kbest(orc, label, P, x_gpu, pd_gpu, out, R, z, forced, terms=3):
    """Parity of a K-best detection with the oracle's `out` on the same
    frames.  x_gpu [B, n] PAM indices and pd_gpu [B] from the GPU; R, z the
    oracle's QR; forced(mask, x) runs the oracle on frames[mask] with x
    forced and returns its fgap.  Returns (eps_FP32, tol, n_mismatch)."""
    x_gpu = np.asarray(x_gpu)
    pd_gpu = np.asarray(pd_gpu, np.float64)
    same = np.all(x_gpu == out["x"], axis=1)
    eps = 0.0
    if same.any():
        bnd = pd_error_bound(R[same], z[same], out["x"][same], P, terms)
        err = np.abs(pd_gpu[same] - out["pd"][same])
        bad = np.nonzero(err > bnd)[0]
        assert bad.size == 0, (f"{label}: FP32 search pd outside the derived bound on {bad.size} frames, "
                               f"e.g. err {err[bad[0]]:.3e} > {bnd[bad[0]]:.3e}")
        eps = float(np.max(err / np.maximum(out["pd"][same], 1e-300)))
    tol = near_tie_tol(eps)
    mism = ~same
    nm = int(mism.sum())
    if nm:
        fg = np.asarray(forced(mism, x_gpu[mism]))
        bad = np.nonzero(fg > tol)[0]
        if bad.size:
            raise AssertionError(f"{label}: {bad.size} of {nm} mismatches are not near ties "
                                 f"(forced-path gaps {np.array2string(fg[bad][:5], precision=3)} > tol {tol:.2e})")
    print(f"{label}: eps_FP32 {eps:.2e}, near-tie tol {tol:.2e}, {nm} of {len(same)} frames differ "
          f"(all near ties)" + (f", forced-path gaps up to {np.max(fg):.2e}" if nm else ""))
    return eps, tol, nm


def check_kbest_run(orc, label, P, K, sym_gpu, pd_gpu, out, R, z, k_sched=None, r2=math.inf, J=1, terms=3):
    """check_kbest for a batched oracle run with one radius for all frames
    (k_sched None, [n] or [B, n])."""
    def forced(mask, xf):
        ks = k_sched
        if ks is not None and np.ndim(ks) == 2:
            ks = ks[mask]
        return orc.kbest(R[mask], z[mask], P, K, k_sched=ks, r2=r2, J=J, force_path=xf)["fgap"]

    return check_kbest(orc, label, P, orc.sym_to_x(np.asarray(sym_gpu), P), pd_gpu, out, R, z, forced, terms)


def check_ml(orc, label, P, sym_gpu, out_sd, H, y, qam, metric_gpu=None):
    """Exact-SD parity: both sides return a maximum-likelihood point, so a
    symbol mismatch is excused only when the FP64 metrics of the two points
    are within the near-tie window of each other (two points tied for ML up
    to FP32 rounding); the window is 1e-5, the floor, since the FP64 metric
    is exact to far below it.  Returns the number of mismatches."""
    s_o = orc.x_to_sym(out_sd[0] if isinstance(out_sd, tuple) else out_sd["x"], P)
    sym_gpu = np.asarray(sym_gpu)
    mism = np.any(sym_gpu != s_o, axis=1)
    nm = int(mism.sum())
    if nm:
        mg = orc.metric(H[mism], y[mism], sym_gpu[mism], qam)
        mo = orc.metric(H[mism], y[mism], s_o[mism], qam)
        rel = np.abs(mg - mo) / np.maximum(mo, 1e-300)
        bad = np.nonzero(rel > NEAR_TIE_FLOOR)[0]
        assert bad.size == 0, f"{label}: {bad.size} of {nm} ML mismatches differ in metric by {rel[bad][:5]}"
    print(f"{label}: {nm} of {len(sym_gpu)} frames differ, all ML ties within {NEAR_TIE_FLOOR:g}")
    return nm


def compare_symbols(sym_gpu, sym_orc, margin, tol, label=""):
    """For trajectory searches (the hybrid with workers) whose result depends
    on every radius update: a mismatch is excused iff one of the oracle's own
    decisions on that frame compared two values within tol.  Returns
    (n_mismatch, n_excused)."""
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

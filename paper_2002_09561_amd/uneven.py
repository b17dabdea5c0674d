"""Uneven batches: frames of different antenna counts and constellations
detected together, each kernel in one persistent launch.

A batch is described by one `mimo_frame_desc` record per frame (shape, PAM
points, survivors K and the offsets of its data in flat arrays); the QR and
K-best kernels pull frames from a device work counter.  K per frame comes
from a table keyed by (antennas, QAM order), normally the autotuner's.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import mimo

DESC_DTYPE = np.dtype([("n_rx", "<i4"), ("n_tx", "<i4"), ("pam", "<i4"), ("K", "<i4"), ("h_off", "<i8"),
                       ("y_off", "<i8"), ("r_off", "<i8"), ("z_off", "<i8"), ("s_off", "<i8")])
assert DESC_DTYPE.itemsize == 56


def k_for(table: dict, n_tx: int, qam: int, default: int = 16) -> int:
    return int(table.get(f"{n_tx}x{qam}", default))


# per-frame limits of the persistent K-best launch (kbest_detect_uneven)
UNEVEN_MAX_TX = 64
UNEVEN_MAX_K = 64
UNEVEN_MAX_CAND = 256


def validate_descriptors(desc: np.ndarray) -> None:
    """Rejects (ValueError) descriptors outside the persistent launches'
    range: pam in {2, 4, 8}, 1 <= K <= 64, K * pam <= 256,
    1 <= n_tx <= min(n_rx, 64), n_rx <= 128.  The kernels skip such frames
    (flag INVALID_FRAME) as well; this check stops them before upload."""
    pam, K, ntx, nrx = (desc[f].astype(np.int64) for f in ("pam", "K", "n_tx", "n_rx"))
    bad = (~np.isin(pam, (2, 4, 8)) | (K < 1) | (K > UNEVEN_MAX_K) | (K * pam > UNEVEN_MAX_CAND) | (ntx < 1)
           | (ntx > UNEVEN_MAX_TX) | (nrx < ntx) | (nrx > 128))
    if bad.any():
        i = int(np.nonzero(bad)[0][0])
        raise ValueError(f"{int(bad.sum())} frame descriptors outside the uneven launch's limits, first: frame {i} "
                         f"(n_rx {nrx[i]}, n_tx {ntx[i]}, pam {pam[i]}, K {K[i]})")


class UnevenBatch:
    """Device-resident uneven batch with its descriptors and output buffers.

    `desc_np` holds the descriptors in frame order.  The device copy `desc` is
    in launch order: most expensive frames first (levels x K x PAM points,
    the K-best's work per frame), so that the persistent launches, which pull
    frames in descriptor order, end on cheap frames instead of waiting on a
    late expensive one.  R, z and sym sit at each frame's own offsets; pd and
    flags are indexed by launch position: entry j belongs to frame order[j]
    (`by_frame` reorders them)."""

    def __init__(self, frames, k_table: dict, device="cuda"):
        B = len(frames)
        self.B = B
        n = 2 * frames.n_tx.astype(np.int64)
        rsz = n * (n + 1) // 2
        desc = np.zeros(B, DESC_DTYPE)
        desc["n_rx"] = frames.n_rx
        desc["n_tx"] = frames.n_tx
        desc["pam"] = [math.isqrt(int(q)) for q in frames.qam]
        desc["K"] = [k_for(k_table, int(m), int(q)) for m, q in zip(frames.n_tx, frames.qam)]
        desc["h_off"] = frames.h_off
        desc["y_off"] = frames.y_off
        desc["r_off"] = np.concatenate([[0], np.cumsum(rsz)[:-1]])
        desc["z_off"] = np.concatenate([[0], np.cumsum(n)[:-1]])
        desc["s_off"] = frames.s_off
        validate_descriptors(desc)
        self.desc_np = desc
        cost = n * desc["K"].astype(np.int64) * desc["pam"].astype(np.int64)
        self.order = np.argsort(-cost, kind="stable")
        self.max_rx = int(frames.n_rx.max())
        self.desc = torch.from_numpy(np.ascontiguousarray(desc[self.order]).view(np.uint8)).to(device)
        self.H = torch.from_numpy(frames.H_flat).to(device)
        self.y = torch.from_numpy(frames.y_flat).to(device)
        self.s_true = torch.from_numpy(frames.s_flat).to(device)
        self.R = torch.empty(int(rsz.sum()), device=device)
        self.z = torch.empty(int(n.sum()), device=device)
        self.sym = torch.empty(int(frames.n_tx.sum()), device=device, dtype=torch.int32)
        self.pd = torch.empty(B, device=device)
        self.flags = torch.empty(B, device=device, dtype=torch.int32)
        self.counter = torch.zeros(2, device=device, dtype=torch.int32)

    def run(self, qr_grid: int = 0, kb_grid: int = 0, stream=None):
        """QR and K-best of every frame: two persistent launches."""
        mimo.qr_preprocess_uneven(self.desc, self.B, self.max_rx, self.H, self.y, self.R, self.z,
                                  self.counter[0:1], grid=qr_grid, stream=stream)
        mimo.kbest_detect_uneven(self.desc, self.B, self.R, self.z, self.sym, self.pd, self.flags,
                                 self.counter[1:2], grid=kb_grid, stream=stream)

    def by_frame(self, t: torch.Tensor) -> np.ndarray:
        """A per-launch-position output (pd, flags) in frame order."""
        out = np.empty(self.B, t.cpu().numpy().dtype)
        out[self.order] = t.cpu().numpy()
        return out

    def symbol_errors(self) -> int:
        return int((self.sym != self.s_true).sum())

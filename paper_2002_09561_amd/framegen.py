"""Seeded synthetic MIMO frames for the flat-fading model y = H s + n.

System model (Sec. III-A, Eq. (1)): H is N x M with i.i.d. CN(0, 1) entries,
s is drawn uniformly from a square QAM alphabet, n is complex white Gaussian
noise.  This module only *produces inputs*; it contains no detection
arithmetic and is the one module shared by the oracle tests and the GPU path.

Conventions (readings of the paper where it is silent):
  * square QAM with P = sqrt(|Omega|) points per real dimension, real
    amplitudes (2i - (P-1)) * c with c = sqrt(3 / (2 (|Omega| - 1))) so that
    E|s|^2 = 1; the QAM index of a symbol is i_re * P + i_im;
  * SNR is Es/N0 per stream: complex noise variance sigma^2 = 10^(-SNR/10)
    per receive antenna (sigma^2 / 2 per real part);
  * a fresh H per frame.
H and y are generated in float64 and stored as complex64; both the oracle and
the GPU path read exactly these complex64 values.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

__all__ = ["Frames", "UnevenFrames", "gen_frames", "gen_uneven", "qam_amplitudes"]


def qam_amplitudes(qam: int) -> np.ndarray:
    """Real PAM amplitudes of a unit-energy square QAM, ascending."""
    P = math.isqrt(qam)
    if P * P != qam or P not in (2, 4, 8):
        raise ValueError(f"unsupported QAM order {qam}")
    c = math.sqrt(3.0 / (2.0 * (qam - 1)))
    return (2.0 * np.arange(P) - (P - 1)) * c


@dataclass
class Frames:
    H: np.ndarray        # [B, N, M] complex64
    y: np.ndarray        # [B, N] complex64
    s_idx: np.ndarray    # [B, M] int32, QAM index i_re * P + i_im
    sigma2: float        # complex noise variance per receive antenna
    n_rx: int
    n_tx: int
    qam: int
    snr_db: float

    @property
    def pam(self) -> int:
        return math.isqrt(self.qam)

    def __len__(self) -> int:
        return self.H.shape[0]


def _rng(seed: int, *tags: int) -> np.random.Generator:
    # Philox is counter-based; the key comes from a SeedSequence over the tags.
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, *[int(t) & 0xFFFFFFFF for t in tags]])
    return np.random.Generator(np.random.Philox(ss))


def _symbols(s_idx: np.ndarray, qam: int) -> np.ndarray:
    P = math.isqrt(qam)
    amp = qam_amplitudes(qam)
    return amp[s_idx // P] + 1j * amp[s_idx % P]


def gen_frames(n_rx: int, n_tx: int, qam: int, snr_db: float, n_frames: int,
               seed: int = 0, snr_idx: int = 0) -> Frames:
    """Generate ``n_frames`` frames of an n_rx x n_tx system at one SNR.

    Deterministic in (seed, n_rx, n_tx, qam, snr_idx): frames are produced in
    whole chunks of 256, each from its own Philox stream keyed by the chunk
    index, so frame i is the same whatever the total count.
    """
    chunk = 256
    if n_tx > n_rx:
        raise ValueError("n_tx must not exceed n_rx")
    qam_amplitudes(qam)  # validates
    sigma2 = 10.0 ** (-snr_db / 10.0)
    H = np.empty((n_frames, n_rx, n_tx), np.complex64)
    y = np.empty((n_frames, n_rx), np.complex64)
    s_idx = np.empty((n_frames, n_tx), np.int32)

    def one(c0):
        c1 = min(n_frames, c0 + chunk)
        g = _rng(seed, n_rx, n_tx, qam, snr_idx, c0 // chunk)
        hr = g.standard_normal((chunk, n_rx, n_tx, 2), dtype=np.float32)
        Hc = (hr[..., 0] + 1j * hr[..., 1]).astype(np.complex64) * np.float32(math.sqrt(0.5))
        si = g.integers(0, qam, size=(chunk, n_tx), dtype=np.int32)
        nr = g.standard_normal((chunk, n_rx, 2))
        noise = (nr[..., 0] + 1j * nr[..., 1]) * math.sqrt(sigma2 / 2.0)
        s = _symbols(si, qam)
        yc = np.matmul(Hc.astype(np.complex128), s[:, :, None])[:, :, 0] + noise
        H[c0:c1] = Hc[: c1 - c0]
        y[c0:c1] = yc[: c1 - c0].astype(np.complex64)
        s_idx[c0:c1] = si[: c1 - c0]

    starts = list(range(0, n_frames, chunk))
    if len(starts) > 1:
        with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1, len(starts))) as ex:
            list(ex.map(one, starts))
    else:
        for c0 in starts:
            one(c0)
    return Frames(H, y, s_idx, sigma2, n_rx, n_tx, qam, float(snr_db))


@dataclass
class UnevenFrames:
    """A batch whose frames differ in antenna count, QAM order and SNR.

    Frame f occupies H_flat[h_off[f] : h_off[f] + n_rx*n_tx] (row-major
    [n_rx][n_tx]) and y_flat[y_off[f] : y_off[f] + n_rx]; symbols occupy
    s_flat[s_off[f] : s_off[f] + n_tx].
    """
    n_rx: np.ndarray     # [B] int32
    n_tx: np.ndarray     # [B] int32
    qam: np.ndarray      # [B] int32
    snr_db: np.ndarray   # [B] float64
    sigma2: np.ndarray   # [B] float64
    h_off: np.ndarray    # [B] int64
    y_off: np.ndarray    # [B] int64
    s_off: np.ndarray    # [B] int64
    H_flat: np.ndarray   # complex64
    y_flat: np.ndarray   # complex64
    s_flat: np.ndarray   # int32

    def __len__(self) -> int:
        return self.n_rx.shape[0]

    def frame(self, f: int):
        N, M = int(self.n_rx[f]), int(self.n_tx[f])
        H = self.H_flat[self.h_off[f]: self.h_off[f] + N * M].reshape(N, M)
        y = self.y_flat[self.y_off[f]: self.y_off[f] + N]
        s = self.s_flat[self.s_off[f]: self.s_off[f] + M]
        return H, y, s


def gen_uneven(n_frames: int, seed: int = 0, antennas=(10, 16, 32, 64),
               qams=(4, 16, 64), snr_range=(8.0, 24.0)) -> UnevenFrames:
    """Mixed batch: M = N drawn uniformly from ``antennas``, |Omega| from
    ``qams``, SNR uniform in ``snr_range`` (continuous, stored per frame)."""
    g = _rng(seed, 0xB00B, n_frames)
    n = g.choice(np.asarray(antennas, np.int32), size=n_frames)
    q = g.choice(np.asarray(qams, np.int32), size=n_frames)
    snr = g.uniform(snr_range[0], snr_range[1], size=n_frames)
    sigma2 = 10.0 ** (-snr / 10.0)
    hsz = (n.astype(np.int64) * n)
    h_off = np.concatenate([[0], np.cumsum(hsz)[:-1]]).astype(np.int64)
    y_off = np.concatenate([[0], np.cumsum(n.astype(np.int64))[:-1]]).astype(np.int64)
    H_flat = np.empty(int(hsz.sum()), np.complex64)
    y_flat = np.empty(int(n.sum()), np.complex64)
    s_flat = np.empty(int(n.sum()), np.int32)
    # one Philox stream per (antenna count, qam) group keeps generation vectorised
    for nv in np.unique(n):
        for qv in np.unique(q):
            sel = np.nonzero((n == nv) & (q == qv))[0]
            if sel.size == 0:
                continue
            gg = _rng(seed, 0xB00C, int(nv), int(qv), n_frames)
            b = sel.size
            hr = gg.standard_normal((b, nv, nv, 2), dtype=np.float32)
            Hc = (hr[..., 0] + 1j * hr[..., 1]).astype(np.complex64) * np.float32(math.sqrt(0.5))
            si = gg.integers(0, qv, size=(b, nv), dtype=np.int32)
            nr = gg.standard_normal((b, nv, 2))
            noise = (nr[..., 0] + 1j * nr[..., 1]) * np.sqrt(sigma2[sel] / 2.0)[:, None]
            yc = np.matmul(Hc.astype(np.complex128), _symbols(si, int(qv))[:, :, None])[:, :, 0] + noise
            for r, f in enumerate(sel):
                H_flat[h_off[f]: h_off[f] + nv * nv] = Hc[r].reshape(-1)
                y_flat[y_off[f]: y_off[f] + nv] = yc[r].astype(np.complex64)
                s_flat[y_off[f]: y_off[f] + nv] = si[r]
    return UnevenFrames(n.astype(np.int32), n.astype(np.int32), q.astype(np.int32), snr, sigma2,
                        h_off, y_off, y_off.copy(), H_flat, y_flat, s_flat)

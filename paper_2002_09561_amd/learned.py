"""Learned per-level survivor counts for K-best / the hybrid's workers.

The paper's hybrid lets workers keep extra nodes whose distance is "very
close" to the selected ones (Sec. VI) without fixing a rule.  Here a small
MLP (4 -> 128 -> 128 -> 1, ReLU) predicts, for every level of a frame, a high
quantile of log2 of the rank that the maximum-likelihood path's prefix takes
among that level's sorted candidates; the detector then keeps
K_t = clamp(ceil(2^(prediction + margin)), k_min, k_max) survivors at level t.

Everything here drives the library's kernels (no arithmetic of its own):
  * training states: frames -> QR -> K-best warm radius -> exact Best-FS SD
    (the hybrid kernel with no workers) -> forced-path K-best rank labels and
    per-level features;
  * training: pinball loss (quantile tau) and Adam, both on the GPU;
  * inference: features -> MLP -> schedule.
Weights are stored as a flat float32 checkpoint with a JSON header.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import struct
import sys
import time

import numpy as np
import torch

from . import mimo
from .framegen import gen_frames

MAGIC = b"MIMOMLP1"
HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(HERE, "weights")


# ------------------------------------------------------------ checkpoint
def init_weights(seed: int = 0) -> np.ndarray:
    """He-normal initialisation of the flat parameter vector."""
    rng = np.random.default_rng(seed)
    H, I = mimo.MLP_HIDDEN, mimo.MLP_IN
    parts = [rng.normal(0, math.sqrt(2.0 / I), H * I), np.zeros(H),
             rng.normal(0, math.sqrt(2.0 / H), H * H), np.zeros(H),
             rng.normal(0, math.sqrt(1.0 / H), H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def save_weights(path: str, w, meta: dict, m=None, v=None, step: int = 0):
    """Checkpoint: MAGIC, u32 header length, JSON header, float32 w [, m, v]."""
    w = np.asarray(w.detach().cpu() if isinstance(w, torch.Tensor) else w, np.float32)
    head = dict(meta)
    head.update(nparam=int(w.size), step=int(step), has_moments=m is not None)
    hb = json.dumps(head, sort_keys=True).encode()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "wb") as fh:
        fh.write(MAGIC)
        fh.write(struct.pack("<I", len(hb)))
        fh.write(hb)
        fh.write(w.tobytes())
        if m is not None:
            for a in (m, v):
                a = np.asarray(a.detach().cpu() if isinstance(a, torch.Tensor) else a, np.float32)
                fh.write(a.tobytes())
    os.replace(tmp, path)


def load_weights(path: str, with_moments: bool = False):
    with open(path, "rb") as fh:
        if fh.read(8) != MAGIC:
            raise ValueError(f"{path}: not a weights checkpoint")
        (hl,) = struct.unpack("<I", fh.read(4))
        meta = json.loads(fh.read(hl))
        npar = meta["nparam"]
        w = np.frombuffer(fh.read(4 * npar), np.float32).copy()
        if with_moments and meta.get("has_moments"):
            m = np.frombuffer(fh.read(4 * npar), np.float32).copy()
            v = np.frombuffer(fh.read(4 * npar), np.float32).copy()
            return torch.from_numpy(w), meta, torch.from_numpy(m), torch.from_numpy(v)
    return torch.from_numpy(w), meta


# ------------------------------------------------------------ states and labels
def training_states(n_tx: int, qam: int, snrs, frames_per_snr: int, seed: int, k_warm: int = 16,
                    k_label: int = 64, sd_budget: int = 200000, chunk: int = 2048, log=print):
    """Per-level (features, log2 rank) pairs from frames whose exact SD run
    certified the ML solution.  Returns X [S, 4] f32, y [S] f32 (GPU) and stats."""
    P = math.isqrt(qam)
    n = 2 * n_tx
    Xs, ys = [], []
    stats = dict(frames=0, certified=0, sd_rounds=0)
    for si, snr in enumerate(snrs):
        for c0 in range(0, frames_per_snr, chunk):
            b = min(chunk, frames_per_snr - c0)
            f = gen_frames(n_tx, n_tx, qam, snr, c0 + b, seed=seed, snr_idx=si)
            H = torch.from_numpy(f.H[c0:]).cuda()
            y = torch.from_numpy(f.y[c0:]).cuda()
            R, z = mimo.qr_preprocess(H, y)
            _, pdw, _ = mimo.kbest_detect(R, z, n_tx, P, k_warm)
            r2 = (pdw * (1.0 + 1e-4)).contiguous()
            sym, pd, flags, ctr = mimo.sd_hybrid_detect(R, z, n_tx, P, 0, 1, radius2=r2, node_budget=sd_budget,
                                                        want_counters=True)
            ok = ((flags & mimo.FLAG_CERTIFIED) != 0) & ((flags & mimo.FLAG_FOUND) != 0)
            rank = mimo.kbest_rank_labels(R, z, n_tx, P, k_label, sym)
            s2 = torch.full((b,), f.sigma2, device="cuda", dtype=torch.float32)
            feat = mimo.prune_features(R, z, s2, n_tx, P)
            sel = ok.nonzero().squeeze(1)
            Xs.append(feat[sel].reshape(-1, 4))
            ys.append(torch.log2(rank[sel].clamp_min(1).float()).reshape(-1))
            stats["frames"] += b
            stats["certified"] += int(ok.sum())
            stats["sd_rounds"] += int(ctr[:, 2].sum())
        log(f"  states: {snr} dB done, {stats['certified']}/{stats['frames']} certified")
    return torch.cat(Xs).contiguous(), torch.cat(ys).contiguous(), stats


def train(X: torch.Tensor, y: torch.Tensor, steps: int = 3000, batch: int = 4096, lr: float = 2e-3,
          tau: float = 0.95, seed: int = 0, log=print, w0=None):
    """Adam on the mean pinball loss with the library's backward kernels."""
    S = X.shape[0]
    w = (torch.from_numpy(init_weights(seed)) if w0 is None else w0.clone()).cuda()
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    ws = torch.empty(mimo.mlp_workspace_bytes(batch), device="cuda", dtype=torch.uint8)
    grad = torch.empty_like(w)
    loss = torch.empty(1, device="cuda")
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    hist = []
    for t in range(1, steps + 1):
        idx = torch.randint(0, S, (batch,), generator=g).cuda()
        xb = X[idx].contiguous()
        yb = y[idx].contiguous()
        # cosine learning-rate decay
        lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * (t - 1) / steps))
        mimo.mlp_loss_grad(w, xb, yb, tau, ws=ws, grad=grad, loss=loss)
        mimo.mlp_adam_step(w, m, v, grad, t, lr_t)
        if t % max(1, steps // 10) == 0 or t == 1:
            hist.append((t, float(loss.item())))
            log(f"  step {t}: pinball loss {hist[-1][1]:.4f}")
    return w, m, v, hist


# ------------------------------------------------------------ inference
def schedule(w, R, z, sigma2, n_tx: int, pam: int, margin: float, k_min: int, k_max: int, flags=None):
    """Per-frame, per-level survivor counts [B, n] int32."""
    B = z.shape[0]
    n = 2 * n_tx
    feat = mimo.prune_features(R, z, sigma2, n_tx, pam)
    ks = mimo.mlp_schedule(w, feat.view(B * n, 4), n, margin, k_min, k_max, flags=flags)
    return ks.view(B, n)


def detect(w, R, z, sigma2, n_tx: int, pam: int, margin: float, k_min: int, k_max: int, beta: float,
           fallback_K: int, out=None, feat=None, ks=None, counters=None):
    """Learned detection: per-level schedule -> scheduled K-best -> plain
    K-best fallback for frames flagged or above the noise bound."""
    B = z.shape[0]
    n = 2 * n_tx
    feat = mimo.prune_features(R, z, sigma2, n_tx, pam, out=feat)
    ks = mimo.mlp_schedule(w, feat.view(B * n, 4), n, margin, k_min, k_max,
                           out=None if ks is None else ks.view(B * n)).view(B, n)
    if out is None:
        out = (torch.empty(B, n_tx, device=z.device, dtype=torch.int32), torch.empty(B, device=z.device),
               torch.empty(B, device=z.device, dtype=torch.int32), None)
    mimo.kbest_detect(R, z, n_tx, pam, k_max, k_sched=ks, out=(out[0], out[1], out[2], counters))
    mimo.kbest_fallback(R, z, n_tx, pam, fallback_K, sigma2, beta, out[:3], counters=counters)
    return out[0], out[1], out[2], ks


def calibrate(w, n_tx, qam, snrs, frames, seed, k_min, plain_K, k_maxes, margins, betas, fixed_ks=(), log=print):
    """Fastest (k_max, margin, beta) whose learned detection makes at most 5%
    more symbol errors than plain K-best (K = plain_K, the setting whose
    errors match the exact SD) on the calibration frames at every SNR.  All
    SNR points run as one batch, as in the benchmark."""
    P = math.isqrt(qam)
    fr = [gen_frames(n_tx, n_tx, qam, snr, frames, seed=seed, snr_idx=si) for si, snr in enumerate(snrs)]
    H = torch.from_numpy(np.concatenate([f.H for f in fr])).cuda()
    Y = torch.from_numpy(np.concatenate([f.y for f in fr])).cuda()
    S = torch.from_numpy(np.concatenate([f.s_idx for f in fr])).cuda()
    s2 = torch.from_numpy(np.repeat(np.array([f.sigma2 for f in fr], np.float32), frames)).cuda()
    R, z = mimo.qr_preprocess(H, Y)

    def per_snr_errors(sym):
        return [int(e) for e in (sym != S).view(len(snrs), frames, -1).sum(dim=(1, 2)).cpu()]

    def timed(fn, reps=3):
        fn()  # warm
        ts = []
        for _ in range(reps):  # median of reps
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return r, sorted(ts)[reps // 2]

    (sp, _, _), t_plain = timed(lambda: mimo.kbest_detect(R, z, n_tx, P, plain_K))
    pe = per_snr_errors(sp)
    log(f"  plain K={plain_K}: errors {pe}, {t_plain * 1e3:.2f} ms")

    def fixed(K, beta):  # ablation: constant K with the same fallback, no network
        sym, pd, fl = mimo.kbest_detect(R, z, n_tx, P, K)
        mimo.kbest_fallback(R, z, n_tx, P, plain_K, s2, beta, (sym, pd, fl))
        return sym, fl

    for K in fixed_ks:
        for beta in betas:
            (sf, ff), t = timed(lambda: fixed(K, beta))
            fe = per_snr_errors(sf)
            fb = float(((ff & mimo.FLAG_LEARNED_FALLBACK) != 0).float().mean())
            ok = all(e <= p * 1.05 for e, p in zip(fe, pe))
            log(f"  ablation fixed K={K} beta {beta:.1f}: errors {fe}, fallback {fb:.4f}, {t * 1e3:.2f} ms"
                f"{'  ok' if ok else ''}")
    best = None
    for km in k_maxes:
        for mg in margins:
            for beta in betas:
                (sl, _, fl, ks), t = timed(lambda: detect(w, R, z, s2, n_tx, P, mg, k_min, km, beta, plain_K))
                le = per_snr_errors(sl)
                fb = float(((fl & mimo.FLAG_LEARNED_FALLBACK) != 0).float().mean())
                ok = all(e <= p * 1.05 for e, p in zip(le, pe))
                log(f"  k_max {km} margin {mg:.2f} beta {beta:.1f}: errors {le}, mean K_t {float(ks.float().mean()):.2f},"
                    f" fallback {fb:.4f}, {t * 1e3:.2f} ms{'  ok' if ok else ''}")
                if ok and (best is None or t < best[5]):
                    best = (km, mg, beta, le, float(ks.float().mean()), t, fb, t_plain, pe)
    return best


def main(argv=None):
    ap = argparse.ArgumentParser(description="train the learned survivor-count MLP on the GPU")
    ap.add_argument("--n-tx", type=int, default=100)
    ap.add_argument("--qam", type=int, default=64)
    ap.add_argument("--snrs", default="20,22,24,26,28")
    ap.add_argument("--frames", type=int, default=1000, help="training frames per SNR")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--tau", type=float, default=0.98)
    ap.add_argument("--k-min", type=int, default=1)
    ap.add_argument("--k-max", type=int, default=64)
    ap.add_argument("--k-label", type=int, default=64)
    ap.add_argument("--plain-K", type=int, default=64, help="plain K-best setting whose errors are matched")
    ap.add_argument("--calib-frames", type=int, default=2000)
    ap.add_argument("--seed", type=int, default=777)
    ap.add_argument("--out", default=None)
    ap.add_argument("--calibrate-only", default=None, help="recalibrate an existing checkpoint in place")
    ap.add_argument("--k-maxes", default="16,32,64", help="calibration grid: survivor caps")
    ap.add_argument("--margins", default="2.0,3.0,3.5,4.0,4.5,5.0", help="calibration grid: margins")
    ap.add_argument("--betas", default="2.0,3.0,4.0,6.0", help="calibration grid: fallback thresholds")
    ap.add_argument("--fixed-ks", default="", help="ablation: constant K values logged beside the grid")
    a = ap.parse_args(argv)
    mimo.load()
    snrs = [float(s) for s in a.snrs.split(",")]
    kms = [int(x) for x in a.k_maxes.split(",")]
    mgs = [float(x) for x in a.margins.split(",")]
    bts = [float(x) for x in a.betas.split(",")]
    fks = [int(x) for x in a.fixed_ks.split(",") if x]
    t0 = time.time()
    if a.calibrate_only:
        w, meta, m, v = load_weights(a.calibrate_only, with_moments=True)
        w = w.cuda()
        cal = calibrate(w, a.n_tx, a.qam, snrs, a.calib_frames, a.seed + 1, a.k_min, a.plain_K,
                        k_maxes=kms, margins=mgs, betas=bts, fixed_ks=fks)
        if cal:
            meta.update(k_max=cal[0], margin=cal[1], beta=cal[2], plain_K=a.plain_K)
            meta["calibration"] = dict(symbol_errors_learned=cal[3], symbol_errors_plain=cal[8], mean_k=cal[4],
                                       learned_ms=cal[5] * 1e3, fallback_fraction=cal[6], plain_ms=cal[7] * 1e3,
                                       frames_per_snr=a.calib_frames)
        for k in ("nparam", "step", "has_moments"):
            meta.pop(k, None)
        save_weights(a.out or a.calibrate_only, w, meta, m, v, step=int(meta.get("steps", 0)))
        print(json.dumps({k: meta[k] for k in meta if k != "loss_history"}))
        return
    X, y, st = training_states(a.n_tx, a.qam, snrs, a.frames, a.seed, k_label=a.k_label)
    yc = y.cpu().numpy()
    print(f"states: {X.shape[0]} from {st['certified']} certified frames ({time.time() - t0:.1f} s); "
          f"rank 1: {np.mean(yc == 0):.4f}, rank > 16: {np.mean(yc > 4):.5f}, max rank {2 ** yc.max():.0f}")
    w, m, v, hist = train(X, y, steps=a.steps, batch=a.batch, lr=a.lr, tau=a.tau, seed=a.seed)
    cal = calibrate(w, a.n_tx, a.qam, snrs, a.calib_frames, a.seed + 1, a.k_min, a.plain_K,
                    k_maxes=kms, margins=mgs, betas=bts, fixed_ks=fks)
    tag = f"{a.n_tx}x{a.n_tx}_{a.qam}qam"
    meta = dict(n_tx=a.n_tx, qam=a.qam, snrs=snrs, frames=a.frames, states=int(X.shape[0]), tau=a.tau,
                k_min=a.k_min, k_label=a.k_label, steps=a.steps, lr=a.lr, seed=a.seed,
                loss_history=hist, plain_K=a.plain_K)
    if cal:
        meta.update(k_max=cal[0], margin=cal[1], beta=cal[2])
        meta["calibration"] = dict(symbol_errors_learned=cal[3], symbol_errors_plain=cal[8], mean_k=cal[4],
                                   learned_ms=cal[5] * 1e3, fallback_fraction=cal[6], plain_ms=cal[7] * 1e3,
                                   frames_per_snr=a.calib_frames)
    else:
        meta.update(k_max=a.k_max, margin=5.0, beta=3.0)
    out = a.out or os.path.join(WEIGHTS_DIR, f"prune_mlp_{tag}.bin")
    save_weights(out, w, meta, m, v, step=a.steps)
    print(json.dumps({k: meta[k] for k in meta if k != "loss_history"}))
    print(f"saved {out} ({time.time() - t0:.1f} s total)")


if __name__ == "__main__":
    main()

"""SNR sweeps of one detector, resumable.

Every finished (configuration, SNR) point is appended to a results file as
one JSON line and flushed to disk; a sweep started again with the same
configuration skips the points the file already holds, so an interrupted
sweep resumes at the next missing point.  Frames are not stored: they are
regenerated from the seed (the generator's chunked Philox streams), keyed
by the SNR itself, so a point's frames do not depend on which other SNRs
the sweep lists.  A line cut short by a crash does not parse and is
ignored; its point runs again.

    python -m paper_2002_09561_amd.sweep --n 16 --qam 16 --detector kbest --K 64 \\
        --snrs 4,8,12,16,20 --frames 10000 --out sweep.jsonl

Detectors (all on the GPU through the library): kbest, kbest_complex,
hybrid, hybrid_complex, sd (exact, the tree spread over a workgroup), zf,
mmse, mrc.  Each point reports bit, symbol and frame errors and the
detection throughput (QR excluded, HIP events).
"""
from __future__ import annotations

import argparse
import json
import os
import time
from typing import Callable

DETECTORS = ("kbest", "kbest_complex", "hybrid", "hybrid_complex", "sd", "zf", "mmse", "mrc")


def config_key(cfg: dict) -> str:
    """Canonical text of a configuration: the same settings give the same key."""
    return json.dumps(cfg, sort_keys=True, separators=(",", ":"))


def load_done(path: str, key: str) -> dict:
    """Points already in the results file for this configuration, by SNR.
    Lines that do not parse (a write cut short) or belong to another
    configuration are passed over; the last record of a point wins."""
    done = {}
    if not os.path.exists(path):
        return done
    with open(path, "r", encoding="utf-8") as f:
        for line in f:
            try:
                rec = json.loads(line)
            except json.JSONDecodeError:
                continue
            if isinstance(rec, dict) and rec.get("key") == key and "snr_db" in rec:
                done[float(rec["snr_db"])] = rec
    return done


def _append(path: str, rec: dict) -> None:
    line = json.dumps(rec, sort_keys=True) + "\n"
    with open(path, "a+", encoding="utf-8") as f:
        # a file whose last line was cut short gets a line break first, so the
        # new record starts a line of its own
        f.seek(0, os.SEEK_END)
        if f.tell() > 0:
            f.seek(f.tell() - 1)
            if f.read(1) != "\n":
                f.write("\n")
        f.write(line)
        f.flush()
        os.fsync(f.fileno())


def run_sweep(cfg: dict, snrs, run_point: Callable[[float], dict], path: str, log=print) -> list:
    """Run the missing points of a sweep; returns the records of all its
    SNRs (loaded or new), in the order given."""
    key = config_key(cfg)
    done = load_done(path, key)
    out = []
    for snr in snrs:
        snr = float(snr)
        if snr in done:
            log(f"{snr:g} dB: in {path}, skipped")
            out.append(done[snr])
            continue
        res = run_point(snr)
        rec = {"key": key, "config": cfg, "snr_db": snr, **res}
        _append(path, rec)
        done[snr] = rec
        out.append(rec)
        log(f"{snr:g} dB: {json.dumps(res, sort_keys=True)}")
    return out


def snr_stream(snr_db: float) -> int:
    """Frame-stream tag of an SNR (tenths of a dB), independent of the list."""
    return int(round(snr_db * 10)) & 0x7FFFFFFF


def gpu_point(cfg: dict, snr_db: float) -> dict:
    """One point on cuda:0: frames, QR, the detector, error counts."""
    import math

    import torch

    from . import mimo
    from .framegen import gen_frames

    n_rx, n_tx, qam = cfg["n_rx"], cfg["n_tx"], cfg["qam"]
    P = math.isqrt(qam)
    det = cfg["detector"]
    f = gen_frames(n_rx, n_tx, qam, snr_db, cfg["frames"], seed=cfg["seed"], snr_idx=snr_stream(snr_db))
    H = torch.from_numpy(f.H).cuda()
    y = torch.from_numpy(f.y).cuda()
    ref = torch.from_numpy(f.s_idx).cuda()
    B = H.shape[0]
    if det == "mmse":
        sig2 = torch.full((B,), float(f.sigma2), device="cuda", dtype=torch.float32)
        R, z = mimo.qr_preprocess_mmse(H, y, sig2)
    elif det != "mrc":
        R, z = mimo.qr_preprocess(H, y)
    extra = {}

    def detect():
        if det == "kbest":
            return mimo.kbest_detect(R, z, n_tx, P, cfg["K"])
        if det == "kbest_complex":
            return mimo.kbest_detect_complex(R, z, n_tx, P, cfg["K"])
        if det in ("hybrid", "hybrid_complex"):
            return mimo.sd_hybrid_detect(R, z, n_tx, P, cfg["workers"], cfg["k_worker"],
                                         complex_levels=(det == "hybrid_complex"))
        if det == "sd":
            return mimo.sd_parallel_detect(R, z, n_tx, P, node_budget=cfg.get("node_budget", 0))
        if det in ("zf", "mmse"):
            return (mimo.linear_detect(R, z, n_tx, P),)
        if det == "mrc":
            return (mimo.mrc_detect(H, y, P),)
        raise ValueError(f"unknown detector {det!r}")

    detect()  # untimed: the first launch of a kernel includes its loading
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    res = detect()
    b.record()
    sym = res[0]
    counts = mimo.error_count(sym, ref, P)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    if det == "sd":
        extra["certified_fraction"] = float((res[2] & mimo.FLAG_CERTIFIED).ne(0).float().mean().item())
    bit_e, sym_e, frm_e = (int(v) for v in counts.tolist())
    return {"frames": B, "symbols": B * n_tx, "bits": B * n_tx * int(round(math.log2(qam))),
            "bit_errors": bit_e, "symbol_errors": sym_e, "frames_in_error": frm_e,
            "ser": sym_e / (B * n_tx), "detect_ms": round(ms, 4),
            "detect_frames_per_s": round(B / (ms * 1e-3), 1), **extra}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, default=None, help="square system: n_rx = n_tx = N")
    ap.add_argument("--n-rx", type=int, default=16)
    ap.add_argument("--n-tx", type=int, default=16)
    ap.add_argument("--qam", type=int, default=16, choices=[4, 16, 64])
    ap.add_argument("--detector", default="kbest", choices=DETECTORS)
    ap.add_argument("--K", type=int, default=64)
    ap.add_argument("--workers", type=int, default=3)
    ap.add_argument("--k-worker", type=int, default=8)
    ap.add_argument("--node-budget", type=int, default=0)
    ap.add_argument("--snrs", default="4,8,12,16,20", help="comma-separated SNRs in dB")
    ap.add_argument("--frames", type=int, default=10000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default="sweep.jsonl")
    args = ap.parse_args(argv)
    n_rx = args.n or args.n_rx
    n_tx = args.n or args.n_tx
    cfg = {"n_rx": n_rx, "n_tx": n_tx, "qam": args.qam, "detector": args.detector,
           "frames": args.frames, "seed": args.seed}
    if args.detector in ("kbest", "kbest_complex"):
        cfg["K"] = args.K
    if args.detector in ("hybrid", "hybrid_complex"):
        cfg.update(workers=args.workers, k_worker=args.k_worker)
    if args.detector == "sd":
        cfg["node_budget"] = args.node_budget
    snrs = [float(s) for s in args.snrs.split(",") if s.strip()]
    t0 = time.perf_counter()
    run_sweep(cfg, snrs, lambda s: gpu_point(cfg, s), args.out)
    print(f"sweep done in {time.perf_counter() - t0:.1f} s -> {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())

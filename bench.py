"""Benchmark: decoded frames/s at matched BER on one MI355X, 100x100 64-QAM.

Workload (one step, the default `c5`): 100x100 complex MIMO, 64-QAM, i.i.d.
Rayleigh H (fresh per frame), SNR 20, 22, 24, 26, 28 dB, 10^4 frames per SNR
(5 x 10^4 frames per step).  Inputs come from the seeded frame generator on
the host and are resident in HBM before timing starts.  One step runs the
whole path for every SNR point: QR preprocessing, detection, the FP64 metric
epilogue and the error counts.

Detectors (all on the same frames):
  learned         per-level state -> MLP survivor schedule -> scheduled K-best
                  -> plain K-best fallback for flagged frames (the headline
                  `value`);
  kbest           plain batched K-best with K = 64, the ladder setting whose
                  errors match the exact sphere decoder ("plain");
  hybrid          the paper's SD-K-best (Best-FS master + K-best workers);
  learned_hybrid  the same hybrid whose workers keep the learned per-level
                  survivor counts (capped at their K_w);
  fixed           ablation: the learned detector's fallback behind a constant K.
An untimed exact-SD leg (hybrid kernel with no workers, warm-started by
K-best) gives the maximum-likelihood reference; the CPU oracle certifies it on
every frame any detector gets wrong or disagrees on, plus a random sample,
and the matched-BER statistics are paired per frame against it.

Other workloads (`--workload`): c2 (16x16 16-QAM, 4-20 dB, plain K-best
K = 64 and the hybrid), c4 (32x32 16-QAM, 12-20 dB, learned vs plain),
uneven (1e5 mixed frames in persistent launches), sdkbest (16x16 64-QAM,
18-28 dB: the SD-K-best and K-best settings of the paper's Sec. VII figures
on the complex-symbol tree, with symbol error rates and visited-node counts
beside the values the paper prints), and train (training steps of the
learned survivor count's network on level states of 32x32 16-QAM frames).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]; prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published FP32 vector peak
PEAK_FP64_VECTOR_TFLOPS = 78.6    # MI355X published FP64 vector peak
PEAK_HBM_GBPS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
WDIR = os.path.join(ROOT, "paper_2002_09561_amd", "weights")

WORKLOADS = {
    "c5": dict(metric="decoded frames/s at matched BER, 100x100 64-QAM, learned vs plain, one MI355X",
               desc="100x100 complex MIMO, 64-QAM, i.i.d. Rayleigh H, SNR 20-28 dB step 2",
               n=100, qam=64, snrs="20,22,24,26,28", frames=10000, K=64, head="learned",
               weights="prune_mlp_100x100_64qam.bin", legs=("kbest", "hybrid", "learned_hybrid")),
    "c2": dict(metric="decoded frames/s, 16x16 16-QAM, plain K-best K=64 and hybrid SD-K-best, one MI355X",
               desc="16x16 complex MIMO, 16-QAM, i.i.d. Rayleigh H, SNR 4-20 dB step 4",
               n=16, qam=16, snrs="4,8,12,16,20", frames=10000, K=64, head="kbest", weights=None,
               legs=("hybrid",)),
    "c4": dict(metric="decoded frames/s at matched BER, 32x32 16-QAM, learned vs plain, one MI355X",
               desc="32x32 complex MIMO, 16-QAM, i.i.d. Rayleigh H, SNR 12-20 dB step 2",
               n=32, qam=16, snrs="12,14,16,18,20", frames=10000, K=64, head="learned",
               weights="prune_mlp_32x32_16qam.bin", legs=("kbest",)),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="c5", choices=["c5", "c2", "c4", "uneven", "sdkbest", "train"])
    p.add_argument("--train-batch", type=int, default=4096, help="states per training step (--workload train)")
    p.add_argument("--frames", type=int, default=0, help="frames per SNR point (0: the workload's)")
    p.add_argument("--snrs", default=None)
    p.add_argument("--detector", default="auto",
                   choices=["auto", "kbest", "learned", "hybrid", "learned_hybrid", "fixed"])
    p.add_argument("--fixed-k", type=int, default=0,
                   help="ablation leg: plain K-best with this K plus the same fallback (0: the learned mean K_t, rounded)")
    p.add_argument("--K", type=int, default=0, help="plain K-best survivors (0: the workload's matched-BER setting)")
    p.add_argument("--workers", type=int, default=3,
                   help="hybrid workers (SD-K-best legs; error counts measured equal for 3 to 15 at 100x100 64-QAM)")
    p.add_argument("--k-worker", type=int, default=8)
    p.add_argument("--hybrid-budget", type=int, default=20000,
                   help="learned hybrid: node expansions per frame (0: none); a frame that reaches it keeps its best "
                        "leaf only if the fallback's bound accepts it, else plain K-best detects it again")
    p.add_argument("--margin", type=float, default=None)
    p.add_argument("--beta", type=float, default=None)
    p.add_argument("--no-compare", action="store_true", help="skip the comparison legs")
    p.add_argument("--no-ml", action="store_true", help="skip the exact-SD reference and matched-BER statistics")
    p.add_argument("--certify-sample", type=int, default=16, help="random frames per SNR certified by the oracle")
    p.add_argument("--cpu-baseline-seconds", type=float, default=12.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="also run a plain device copy of this size (counter calibration)")
    p.add_argument("--seed", type=int, default=2020)
    p.add_argument("--no-graph", action="store_true", help="skip the hipGraph-replayed timing")
    p.add_argument("--uneven-frames", type=int, default=100000)
    p.add_argument("--no-extra", action="store_true",
                   help="c5: skip the uneven-batch and 32x32 figures added to the line")
    return p.parse_args()


# ------------------------------------------------------------ algorithmic work
def qr_flops(N, M):
    """Cholesky QR of [H | y] (C = M + 1 columns) in FP64, 8 real flops per
    complex multiply-add: the Gram matrix's upper triangle, C (C + 1) / 2
    entries over N rows, then Cholesky step k updating the (C-1-k)(C-k)/2
    upper entries of the trailing Schur complement."""
    C = M + 1
    gram = 8.0 * N * C * (C + 1) / 2
    k = np.arange(M)
    chol = float(np.sum(8.0 * (C - 1 - k) * (C - k) / 2))
    return gram + chol


def kbest_flops_from_counts(cnt, P):
    """cnt[t] = survivors expanded at depth t (t symbols fixed): each costs t
    FMAs for its centre and 2 FMAs per child."""
    t = np.arange(cnt.shape[0])
    return float(np.sum(cnt * (2.0 * t + 4.0 * P)))


def kbest_bytes_per_frame(n, M, sched=False):
    """Algorithmic HBM bytes of one frame's K-best: R (packed) and z read
    once, the schedule read once if any, symbols, pd and flags written."""
    return 4.0 * (n * (n + 1) // 2 + n) + (4.0 * n if sched else 0.0) + 4.0 * M + 8.0


def plain_counts(n, P, K):
    cnt = np.empty(n)
    c = 1
    for t in range(n):
        cnt[t] = c
        c = min(K, c * P)
    return cnt


def sched_counts(ks: np.ndarray, P: int) -> np.ndarray:
    """ks [B, n] by level -> survivors expanded at each depth, summed over frames."""
    B, n = ks.shape
    tot = np.zeros(n)
    c = np.ones(B)
    for t in range(n):
        tot[t] = c.sum()
        c = np.minimum(ks[:, n - 1 - t], c * P)
    return tot


def alu_roofline(flops, ms):
    achieved = flops / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 5), "avg_launch_ms": round(ms, 4),
            "algorithmic_flops_per_launch": flops}


def hbm_roofline(nbytes, ms):
    achieved = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 5), "avg_launch_ms": round(ms, 4),
            "algorithmic_bytes_per_launch": nbytes}


def kernel_source_hash(name):
    h = hashlib.sha256()
    for f in ("common.hpp", name):
        h.update(open(os.path.join(ROOT, "paper_2002_09561_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def clopper_pearson(k: int, n: int, alpha: float = 0.05):
    """Exact two-sided binomial confidence interval for k successes in n."""
    from scipy.stats import beta

    lo = 0.0 if k == 0 else float(beta.ppf(alpha / 2, k, n - k + 1))
    hi = 1.0 if k == n else float(beta.ppf(1 - alpha / 2, k + 1, n - k))
    return [lo, hi]


# ------------------------------------------------------------ CPU baseline (the FP64 oracle)
def cpu_baseline(frames, W, head, K, meta, budget_s, legs, workers=3, k_worker=8):
    """The FP64 oracle (C, OpenMP over frames) on bounded samples of the
    step's own frames: the headline detector's pipeline (QR, then the
    learned detector or plain K-best, then the metric), and the comparison
    detectors for half the time each."""
    import oracle

    f = frames[0]
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    chunk = max(16, 2 * cores)
    w64 = None if W is None else W.cpu().numpy().astype(np.float64)

    def detector(name):
        if name == "learned":
            return lambda R, z: oracle.learned_detect(R, z, f.pam, f.sigma2, w64, meta["margin"], meta["k_min"],
                                                      meta["k_max"], meta["beta"], K)["x"]
        if name == "kbest":
            return lambda R, z: oracle.kbest(R, z, f.pam, K)["x"]
        if name == "hybrid":
            return lambda R, z: oracle.hybrid(R, z, f.pam, workers, k_worker)["x"]
        return None

    def timed(name, seconds):
        fn = detector(name)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds and done + chunk <= len(f):
            H, y = f.H[done:done + chunk], f.y[done:done + chunk]
            R, z, _ = oracle.qr(H, y)
            oracle.metric(H, y, oracle.x_to_sym(fn(R, z), f.pam), f.qam)
            done += chunk
        dt = time.perf_counter() - t0
        return done, dt

    done, dt = timed(head, budget_s)
    what = {"learned": "learned detector (features, MLP, scheduled K-best, K=%d fallback)" % K,
            "kbest": f"K-best K={K}"}[head]
    out = {"value": round(done / dt, 2), "unit": "frames/s", "cores": cores, "kind": "oracle",
           "sample": f"{done} frames of {f.n_rx}x{f.n_tx} {f.qam}-QAM at {f.snr_db:g} dB (the first frames of the "
                     f"GPU step): FP64 QR + {what} + metric, {dt:.1f} s wall on {cores} threads"}
    other = {}
    for leg in legs:
        if detector(leg) is None:
            continue
        d, t = timed(leg, budget_s / 2)
        other[leg] = {"frames_per_s": round(d / t, 2), "frames": d, "seconds": round(t, 1)}
        if leg == "hybrid":
            other[leg]["detector"] = f"SD-K-best, {workers} workers x {k_worker} survivors"
    if other:
        out["legs"] = other
    return out


def certify_ml(idx, frames, B, P, qam, budget=20_000_000):
    """The oracle's maximum-likelihood points of the frames idx (positions in
    the step's batch): QR, K-best K = 64 for a warm radius, then the Best-FS
    SD certifying the exact ML point inside it.  Returns (QAM indices
    [len(idx), M], certified flags)."""
    import oracle

    H = np.concatenate([frames[i // B].H[i % B][None] for i in idx])
    y = np.concatenate([frames[i // B].y[i % B][None] for i in idx])
    R, z, _ = oracle.qr(H, y)
    kb = oracle.kbest(R, z, P, 64)
    x, _, fl, _ = oracle.sesd(R, z, P, r2=kb["pd"] * (1 + 1e-12), x_init=kb["x"], budget=budget)
    return oracle.x_to_sym(x, P), (fl & oracle.CERTIFIED) != 0, H, y


# ------------------------------------------------------------ uneven batches
def uneven_run(args):
    """Config: 1e5 frames, M = N drawn from {10, 16, 32, 64}, QAM from {4, 16,
    64}, SNR uniform 8-24 dB; QR and K-best each in one persistent launch,
    K per class and grids from the autotuner's cache; the step is captured in
    a hipGraph and replayed.  Returns the result line as a dict."""
    import torch

    from paper_2002_09561_amd import autotune, mimo, uneven
    from paper_2002_09561_amd.framegen import gen_uneven
    from paper_2002_09561_amd.graph import CapturedStep

    torch.cuda.set_device(0)
    mimo.load()
    tune = autotune.load() or autotune.load("gfx950")
    if tune is None:
        raise SystemExit("no autotuner cache: run python -m paper_2002_09561_amd.autotune")
    fr = gen_uneven(args.uneven_frames, seed=args.seed)
    ub = uneven.UnevenBatch(fr, tune["k_table"])
    step = lambda: ub.run(qr_grid=tune["qr_grid"], kb_grid=tune["kbest_grid"])
    g = CapturedStep(step, warmup=max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a.record()
    mimo.qr_preprocess_uneven(ub.desc, ub.B, ub.max_rx, ub.H, ub.y, ub.R, ub.z, ub.counter[0:1], tune["qr_grid"])
    b.record()
    mimo.kbest_detect_uneven(ub.desc, ub.B, ub.R, ub.z, ub.sym, ub.pd, ub.flags, ub.counter[1:2], tune["kbest_grid"])
    c.record()
    torch.cuda.synchronize()
    classes = {}
    for m, q in zip(fr.n_tx, fr.qam):
        classes[f"{m}x{q}"] = classes.get(f"{m}x{q}", 0) + 1
    out = {"metric": "decoded frames/s, uneven batch (1e5 mixed frames), one MI355X",
           "value": round(ub.B * args.steps / dt, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "uneven: M = N in {10,16,32,64}, QAM in {4,16,64}, SNR U[8,24] dB",
                      "frames": ub.B, "classes": classes, "k_table": tune["k_table"], "qr_grid": tune["qr_grid"],
                      "kbest_grid": tune["kbest_grid"], "graph": True},
           "kernel_ms": {"qr_uneven": round(a.elapsed_time(b), 4), "kbest_uneven": round(b.elapsed_time(c), 4)},
           "symbol_error_rate": float(ub.symbol_errors()) / int(fr.n_tx.sum())}
    return out


# ------------------------------------------------------------ SD-K-best on the complex-symbol tree
# The points the paper prints for 16x16 64-QAM (Sec. VII, the SD-K-best versus
# K-best figures: symbol error rate, and visited nodes per thread, at 18-28 dB;
# 1 master + 19 K-best worker threads on a CPU).  Context for the measured
# values, not a target: the paper's threads run asynchronously, its SNR scale
# is not stated, and this kernel has at most 15 workers.
PAPER_SDKBEST_16X16_64QAM = {
    "snr_db": [18, 20, 22, 24, 26, 28],
    "symbol_error_rate": {
        "kbest_k10": [0.038, 0.015, 0.008, 0.0043, 0.0029, 0.0011],
        "kbest_k32": [0.005435, 0.0024, 0.001, 0.0007, 0.0005, 0.0003],
        "sdkbest_k1": [0.028, 0.009, 0.003, 0.00099, 0.00045, 0.00014],
        "sdkbest_k2": [0.011, 0.003, 0.0009, 0.000326, 0.000055, 0.000027],
        "sdkbest_k6": [0.0027, 0.0005513, 0.00023, 0.0001, 0.000044, 0.000018],
        "sdkbest_k8": [0.00244, 0.00028, 0.00013, 0.00007, 0.000034, 0.000019]},
    "visited_nodes_per_thread": {
        "kbest_k10": [151] * 6, "kbest_k32": [481] * 6,
        "sdkbest_k1": [106, 64, 39, 24, 18, 14], "sdkbest_k2": [135, 88, 56, 40, 30, 25],
        "sdkbest_k6": [247, 162, 103, 71, 51, 40], "sdkbest_k8": [297, 193, 123, 84, 57, 43]},
    "threads": "1 master + 19 K-best workers"}


def sdkbest_main(args):
    """16x16 64-QAM, SNR 18-28 dB step 2 (10^4 frames per SNR by default), on
    the complex-symbol tree (64 children per node): K-best with K = 10 and 32
    and the hybrid SD-K-best with 15 workers keeping k in {1, 2, 6, 8}; the
    exact parallel SD warm-started by K-best K = 32 is the ML reference.  The
    timed step (`value`) is QR preprocessing + SD-K-best k = 8 over the whole
    sweep; every leg's detection is timed on its own with HIP events.
    Visited nodes = node expansions (the master's plus every survivor a worker
    expands); per thread = that over the 1 + 15 waves of a frame."""
    import torch

    from paper_2002_09561_amd import mimo
    from paper_2002_09561_amd.framegen import gen_frames

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mimo.load()
    M, QAM, P, W = 16, 64, 8, 15
    snrs = [float(x) for x in (args.snrs or "18,20,22,24,26,28").split(",")]
    B = args.frames or 10000
    frames = [gen_frames(M, M, QAM, s, B, seed=args.seed, snr_idx=i) for i, s in enumerate(snrs)]
    NB = B * len(snrs)
    H = torch.from_numpy(np.concatenate([f.H for f in frames])).cuda()
    Y = torch.from_numpy(np.concatenate([f.y for f in frames])).cuda()
    s_true = np.concatenate([f.s_idx for f in frames])
    n = 2 * M
    R = torch.empty(NB, n * (n + 1) // 2, device="cuda")
    z = torch.empty(NB, n, device="cuda")
    budget = 1_000_000

    def outputs():
        return (torch.empty(NB, M, device="cuda", dtype=torch.int32), torch.empty(NB, device="cuda"),
                torch.empty(NB, device="cuda", dtype=torch.int32),
                torch.empty(NB, 4, device="cuda", dtype=torch.int64))

    def kb(K):
        return lambda out: mimo.kbest_detect_complex(R, z, M, P, K, want_counters=True, out=out)

    def sdkb(k):
        return lambda out: mimo.sd_hybrid_detect(R, z, M, P, W, k, node_budget=budget, want_counters=True,
                                                 out=out, complex_levels=True)

    legs = [("kbest_k10", kb(10), 1), ("kbest_k32", kb(32), 1)] + [(f"sdkbest_k{k}", sdkb(k), 1 + W)
                                                                   for k in (1, 2, 6, 8)]

    def event_ms(fn, reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    qr = lambda: mimo.qr_preprocess(H, Y, out=(R, z, None))
    qr()
    torch.cuda.synchronize()
    res, outs = {}, {}
    for name, fn, threads in legs:
        out = outputs()
        for _ in range(max(1, args.warmup)):
            fn(out)
        ms = event_ms(lambda: fn(out), max(1, args.steps))
        sym, flags, ctr = out[0].cpu().numpy(), out[2].cpu().numpy(), out[3].cpu().numpy()
        outs[name] = out
        wrong = (sym != s_true).reshape(len(snrs), B, M)
        nodes = ctr[:, 0].reshape(len(snrs), B).astype(np.float64)
        res[name] = {"detect_ms": round(ms, 3), "detect_frames_per_s": round(NB / ms * 1e3, 1),
                     "symbol_error_rate": [float(x) for x in wrong.mean(axis=(1, 2))],
                     "symbol_errors": [int(x) for x in wrong.sum(axis=(1, 2))],
                     "visited_nodes_mean": [round(float(x), 2) for x in nodes.mean(axis=1)],
                     "visited_nodes_per_thread": [round(float(x) / threads, 2) for x in nodes.mean(axis=1)],
                     "budget_exhausted_frames": int(np.count_nonzero(flags & mimo.FLAG_BUDGET_EXHAUSTED))}
        print(f"# {name}: {ms:.2f} ms, SER {res[name]['symbol_error_rate']}", file=sys.stderr, flush=True)

    # ML reference: the exact parallel SD inside K-best K = 32's leaf metric
    r2 = (outs["kbest_k32"][1] * (1.0 + 1e-4)).contiguous()
    ml = outputs()
    ml_ms = event_ms(lambda: mimo.sd_parallel_detect(R, z, M, P, radius2=r2, node_budget=20_000_000,
                                                     want_counters=True, out=ml), 1)
    sym_ml, fl_ml = ml[0].cpu().numpy(), ml[2].cpu().numpy()
    wrong_ml = (sym_ml != s_true).reshape(len(snrs), B, M)
    ml_ref = {"method": "exact parallel SD (sd_parallel_detect) inside K-best K = 32's leaf metric x (1 + 1e-4)",
              "detect_ms": round(ml_ms, 3), "symbol_error_rate": [float(x) for x in wrong_ml.mean(axis=(1, 2))],
              "symbol_errors": [int(x) for x in wrong_ml.sum(axis=(1, 2))],
              "certified_fraction": float(np.mean((fl_ml & mimo.FLAG_CERTIFIED) != 0))}

    # the timed step: QR + SD-K-best k = 8 over the sweep
    head = outputs()
    step = lambda: (qr(), legs[-1][1](head))
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    qr_ms = event_ms(qr, max(1, args.steps))
    out = {"metric": "decoded frames/s, 16x16 64-QAM SD-K-best on the complex-symbol tree (15 workers x 8), "
                     "one MI355X",
           "value": round(NB * args.steps / dt, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "16x16 complex MIMO, 64-QAM, i.i.d. Rayleigh H, SNR 18-28 dB step 2, "
                                  "complex-symbol tree", "snr_db": snrs, "frames_per_snr": B, "workers": W,
                      "node_budget": budget},
           "qr_ms": round(qr_ms, 3), "legs": res, "ml_reference": ml_ref,
           "paper_context": PAPER_SDKBEST_16X16_64QAM}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------ training the learned survivor count
# algorithmic FP32 flops per state of one training step: forward (4x128,
# 128x128, 128x1 products), the backward delta through W2, and the weight
# gradients (two flops per multiply-add; biases one add each)
MLP_FWD_FLOPS = 2 * (4 * 128 + 128 * 128 + 128)
MLP_TRAIN_FLOPS = MLP_FWD_FLOPS + 2 * 128 * 128 + 2 * (4 * 128 + 128 * 128 + 128) + (128 + 128 + 1)


def train_main(args):
    """One step = the pinball-loss gradient of a batch of level states
    (prune_mlp_loss_grad: per-state forward and backward, then the weight
    gradients as products over the states on the matrix cores) and an Adam
    step.  The states are those the learned detector is trained on: the
    per-level features of 32x32 16-QAM frames at 12-20 dB, labelled by the
    GPU's exact SD (learned.training_states), shuffled once and resident in
    HBM; step i takes the next contiguous batch."""
    import torch

    from paper_2002_09561_amd import learned, mimo

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mimo.load()
    M, QAM, snrs = 32, 16, [12.0, 14.0, 16.0, 18.0, 20.0]
    frames = args.frames or 1000
    t_gen = time.perf_counter()
    X, y, st = learned.training_states(M, QAM, snrs, frames, args.seed, log=lambda *a, **k: None)
    S, bs = X.shape[0], args.train_batch
    if S < 2 * bs:
        raise SystemExit(f"{S} states for batches of {bs}: raise --frames")
    g = torch.Generator(device="cpu")
    g.manual_seed(args.seed)
    perm = torch.randperm(S, generator=g).cuda()
    X, y = X[perm].contiguous(), y[perm].contiguous()
    w = torch.from_numpy(learned.init_weights(args.seed)).cuda()
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    ws = torch.empty(mimo.mlp_workspace_bytes(bs), device="cuda", dtype=torch.uint8)
    grad, loss = torch.empty_like(w), torch.empty(1, device="cuda")
    nb = S // bs
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    ev = {"loss_grad": [], "adam": []}
    state = {"t": 0}

    def step(record):
        i = state["t"] % nb
        state["t"] += 1
        xb, yb = X[i * bs:(i + 1) * bs], y[i * bs:(i + 1) * bs]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)] if record else None
        if record:
            e[0].record()
        mimo.mlp_loss_grad(w, xb, yb, 0.95, ws=ws, grad=grad, loss=loss)
        if record:
            e[1].record()
        mimo.mlp_adam_step(w, m, v, grad, state["t"], 1e-3)
        if record:
            e[2].record()
            ev["loss_grad"].append((e[0], e[1]))
            ev["adam"].append((e[1], e[2]))

    for _ in range(max(1, args.warmup)):
        step(False)
    loss0 = float(loss.item())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms = {k: sum(a.elapsed_time(b) for a, b in v) / len(v) for k, v in ev.items()}
    flops = MLP_TRAIN_FLOPS * bs
    achieved = flops / (kms["loss_grad"] * 1e-3) / 1e12
    out = {"metric": "MLP training states/s (pinball-loss gradient + Adam), 32x32 16-QAM level states, one MI355X",
           "value": round(bs * args.steps / dt, 1), "unit": "states/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "MLP 4-128-128-1 training steps on 32x32 16-QAM level states, 12-20 dB",
                      "states": S, "batch": bs, "certified_frames": st["certified"], "frames": st["frames"]},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_VECTOR_TFLOPS,
                        "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": None,
                        "kernel": "prune_mlp_loss_grad (mlp_backward_states, mlp_grad_tiles, mlp_grad_sum)",
                        "avg_launch_ms": round(kms["loss_grad"], 4),
                        "algorithmic_flops_per_launch": flops},
           "kernel_avg_ms": {k: round(x, 4) for k, x in kms.items()},
           "loss": {"after_warmup": loss0, "end": float(loss.item())}, "setup_s": round(t_gen, 1)}
    if not args.no_cpu_baseline:
        import oracle

        n = min(bs, 2048)
        w64 = w.cpu().numpy().astype(np.float64)
        x64, y64 = X[:n].cpu().numpy().astype(np.float64), y[:n].cpu().numpy().astype(np.float64)
        done, tc = 0, time.perf_counter()
        while time.perf_counter() - tc < args.cpu_baseline_seconds:
            oracle.mlp_loss_grad(w64, x64, y64, 0.95)
            done += n
        tc = time.perf_counter() - tc
        out["cpu_baseline"] = {"value": round(done / tc, 1), "unit": "states/s", "cores": 1, "kind": "oracle",
                               "sample": f"the oracle's FP64 loss and gradient on {n} of the states, repeated for "
                                         f"{tc:.1f} s (single-threaded C)"}
    print(json.dumps(out), flush=True)


# ------------------------------------------------------------ the sweep workloads
def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on several GPUs are not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.workload == "uneven":
        print(json.dumps(uneven_run(args)), flush=True)
        return
    if args.workload == "sdkbest":
        return sdkbest_main(args)
    if args.workload == "train":
        return train_main(args)
    out = sweep_run(args)
    if args.workload == "c5" and not args.no_extra:
        out["other_workloads"] = extra_workloads(args)
    print(json.dumps(out), flush=True)


def extra_workloads(args):
    """Two more configurations in the same run, throughput and errors only:
    the uneven batch (10^5 mixed frames, persistent launches, graph-replayed)
    and 32x32 16-QAM (learned against plain K-best and the ablation; no
    exact-SD reference, CPU baseline or graph replay).  A failure is reported
    in place of the numbers rather than ending the run."""
    import copy

    res = {}
    a = copy.copy(args)
    a.workload, a.steps, a.warmup = "uneven", max(3, args.steps), 1
    try:
        u = uneven_run(a)
        res["uneven"] = {k: u[k] for k in ("metric", "value", "unit", "steps", "ms_per_step", "kernel_ms",
                                           "symbol_error_rate")}
        res["uneven"]["workload"] = u["config"]["workload"]
    except Exception as e:  # noqa: BLE001 - reported in the line
        res["uneven"] = {"error": repr(e)}
    a = copy.copy(args)
    a.workload, a.steps, a.warmup = "c4", 3, 1
    a.no_ml, a.no_cpu_baseline, a.no_graph, a.copy_probe_mib = True, True, True, 0
    a.frames, a.snrs, a.K, a.fixed_k, a.detector, a.margin, a.beta = 0, None, 0, 0, "auto", None, None
    try:
        c = sweep_run(a)
        res["c4"] = {k: c[k] for k in ("metric", "value", "unit", "steps", "ms_per_step", "kernel_avg_ms", "errors")}
        res["c4"]["workload"] = c["config"]["workload"]
        for leg in ("plain_kbest", "ablation_fixed_k"):
            if leg in c:
                res["c4"][leg] = {k: c[leg][k] for k in ("detector", "frames_per_s", "symbol_errors") if k in c[leg]}
    except Exception as e:  # noqa: BLE001
        res["c4"] = {"error": repr(e)}
    return res


def sweep_run(args):
    """The c5 / c2 / c4 workloads: frames over an SNR sweep, the headline
    detector timed per step, the comparison legs, the exact-SD reference and
    matched-BER statistics, the CPU baseline.  Returns the result line as a
    dict."""
    import torch

    from paper_2002_09561_amd import learned, mimo
    from paper_2002_09561_amd.framegen import gen_frames

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    mimo.load()
    wl = WORKLOADS[args.workload]
    N_RX = N_TX = M = wl["n"]
    QAM = wl["qam"]
    P = math.isqrt(QAM)
    n = 2 * M
    snrs = [float(s) for s in (args.snrs or wl["snrs"]).split(",")]
    B = args.frames or wl["frames"]
    K = args.K or wl["K"]
    weights = os.path.join(WDIR, wl["weights"]) if wl["weights"] else None
    det = args.detector
    if det == "auto":
        det = wl["head"] if (wl["head"] != "learned" or (weights and os.path.exists(weights))) else "kbest"

    # ---------------- inputs (host generation, then resident in HBM): one batch of
    # all SNR points, frame i of SNR point j at index j * B + i
    t_gen = time.perf_counter()
    frames = [gen_frames(N_RX, N_TX, QAM, s, B, seed=args.seed, snr_idx=i) for i, s in enumerate(snrs)]
    NB = B * len(snrs)
    H = torch.from_numpy(np.concatenate([f.H for f in frames])).cuda()
    Y = torch.from_numpy(np.concatenate([f.y for f in frames])).cuda()
    S_true = torch.from_numpy(np.concatenate([f.s_idx for f in frames])).cuda()
    SIG2 = torch.from_numpy(np.repeat(np.array([f.sigma2 for f in frames], np.float32), B)).cuda()
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    w, meta = None, {}
    if weights and os.path.exists(weights):
        w, meta = learned.load_weights(weights)
        w = w.cuda()
    margin = args.margin if args.margin is not None else float(meta.get("margin", 4.0))
    beta = args.beta if args.beta is not None else float(meta.get("beta", 3.0))
    k_min, k_max = int(meta.get("k_min", 1)), int(meta.get("k_max", 64))
    meta_run = {"margin": margin, "beta": beta, "k_min": k_min, "k_max": k_max}

    # ---------------- preallocated buffers (nothing is allocated in the timed loop)
    o = dict(R=torch.empty(NB, n * (n + 1) // 2, device="cuda"), z=torch.empty(NB, n, device="cuda"),
             sym=torch.empty(NB, M, device="cuda", dtype=torch.int32), pd=torch.empty(NB, device="cuda"),
             flags=torch.empty(NB, device="cuda", dtype=torch.int32),
             metric=torch.empty(NB, device="cuda", dtype=torch.float64),
             counts=torch.zeros(len(snrs), 3, device="cuda", dtype=torch.int64),
             feat=torch.empty(NB, n, 4, device="cuda"), ks=torch.empty(NB, n, device="cuda", dtype=torch.int32))
    stream = torch.cuda.current_stream()
    ev = {}
    side = torch.cuda.Stream()  # default priority

    def timed(tag, record, fn, st=None):
        if not record:
            return fn()
        st = st or stream
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn()
        b.record(st)
        ev.setdefault(tag, []).append((a, b))

    def fallback_and_metric(record, out3):
        """The fallback's decision first; then the fallback (latency-bound, few
        frames) is launched, and the metric of the frames that keep their first
        detection runs beside it on a side stream (launched second, so that the
        fallback's frames take their wave slots first, in a replayed graph too);
        the re-detected frames' metric follows.  The two kernels touch
        different frames' symbols."""
        fb = mimo.FLAG_LEARNED_FALLBACK
        mimo.kbest_fallback_mark(M, SIG2, beta, out3)
        cur = torch.cuda.current_stream()
        side.wait_stream(cur)
        timed("fallback", record, lambda: mimo.kbest_fallback(o["R"], o["z"], M, P, K, SIG2, beta, out3), st=cur)
        with torch.cuda.stream(side):
            timed("metric", record, lambda: mimo.metric_select(H, Y, o["sym"], P, o["flags"], fb, 0, o["metric"]),
                  st=side)
        cur.wait_stream(side)
        timed("metric_fb", record, lambda: mimo.metric_select(H, Y, o["sym"], P, o["flags"], fb, fb, o["metric"]),
              st=cur)

    fixed_k = args.fixed_k

    def schedule(record):
        timed("features", record, lambda: mimo.prune_features(o["R"], o["z"], SIG2, M, P, out=o["feat"]))
        timed("mlp", record, lambda: mimo.mlp_schedule(w, o["feat"].view(NB * n, 4), n, margin, k_min, k_max,
                                                       out=o["ks"].view(NB * n)))

    def step(detector, record):
        out3 = (o["sym"], o["pd"], o["flags"], None)
        timed("qr", record, lambda: mimo.qr_preprocess(H, Y, out=(o["R"], o["z"], None)))
        if detector == "kbest":
            timed("kbest", record, lambda: mimo.kbest_detect(o["R"], o["z"], M, P, K, out=out3))
        elif detector == "fixed":  # ablation: the learned detector without its network
            timed("kbest", record, lambda: mimo.kbest_detect(o["R"], o["z"], M, P, fixed_k, out=out3))
            fallback_and_metric(record, out3)
        elif detector == "hybrid":
            timed("hybrid", record, lambda: mimo.sd_hybrid_detect(o["R"], o["z"], M, P, args.workers, args.k_worker,
                                                                  out=out3))
        elif detector == "learned_hybrid":
            schedule(record)
            timed("hybrid", record, lambda: mimo.sd_hybrid_detect(o["R"], o["z"], M, P, args.workers, args.k_worker,
                                                                  k_sched=o["ks"], node_budget=args.hybrid_budget,
                                                                  out=out3))
            fallback_and_metric(record, out3)
        else:
            schedule(record)
            timed("kbest", record, lambda: mimo.kbest_detect(o["R"], o["z"], M, P, k_max, k_sched=o["ks"],
                                                             out=out3))
            fallback_and_metric(record, out3)
        if detector in ("kbest", "hybrid"):
            timed("metric", record, lambda: mimo.metric(H, Y, o["sym"], P, out=o["metric"]))
        for i in range(len(snrs)):  # per-SNR error counts
            sl = slice(i * B, (i + 1) * B)
            timed("errors", record, lambda: mimo.error_count(o["sym"][sl], S_true[sl], P, counts=o["counts"][i]))

    syms = {}

    def run(detector, record):
        for _ in range(args.warmup):
            step(detector, False)
        o["counts"].zero_()
        ev.clear()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(detector, record)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        counts = o["counts"].cpu().numpy() // max(1, args.steps)
        kavg = {k: float(np.mean([a.elapsed_time(b) for a, b in v])) for k, v in ev.items()}
        syms[detector] = o["sym"].clone()
        extra = {}
        if detector in ("learned", "learned_hybrid", "fixed"):
            fl = o["flags"].cpu().numpy()
            extra["fallback_fraction"] = float(((fl & mimo.FLAG_LEARNED_FALLBACK) != 0).mean())
        if detector in ("learned", "learned_hybrid"):
            ks = o["ks"].cpu().numpy()
            extra["mean_k_t"] = float(ks.mean())
            extra["ks"] = ks
        if detector == "learned_hybrid" and args.hybrid_budget > 0:
            # the fallback rewrites the flags of the frames it detects again:
            # the budget's share from one more (untimed) hybrid call
            fb = mimo.sd_hybrid_detect(o["R"], o["z"], M, P, args.workers, args.k_worker, k_sched=o["ks"],
                                       node_budget=args.hybrid_budget)[2]
            extra["budget_exhausted_fraction"] = float(((fb & mimo.FLAG_BUDGET_EXHAUSTED) != 0).float().mean())
        return dt, counts, kavg, extra

    frames_per_step = B * len(snrs)
    not_detect = ("qr", "metric", "metric_fb", "errors")

    # ---------------- headline detector (kernel events recorded)
    dt, counts, kavg, extra = run(det, True)
    fps = frames_per_step * args.steps / dt
    dom = max(kavg, key=kavg.get)  # dominant kernel and its roofline
    roofline = None
    if dom == "qr":
        flops, src, kname = qr_flops(N_RX, N_TX) * NB, "qr.hip", "qr_kernel"
        achieved = flops / (kavg[dom] * 1e-3) / 1e12
        traffic = None
        if os.path.exists(TRAFFIC_FILE):
            ent = json.load(open(TRAFFIC_FILE)).get(kname)
            if ent and ent.get("source_hash") == kernel_source_hash(src) and ent.get("frames") == NB:
                traffic = ent.get("bytes_per_launch")
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP64_VECTOR_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_VECTOR_TFLOPS, 4), "traffic": traffic,
                    "kernel": kname, "avg_launch_ms": round(kavg[dom], 4), "algorithmic_flops_per_launch": flops}
    elif dom == "kbest" and det == "kbest":
        roofline = dict(alu_roofline(kbest_flops_from_counts(plain_counts(n, P, K) * NB, P), kavg["kbest"]),
                        traffic=None, kernel="kbest_reg_kernel")

    det_ms = sum(v for k, v in kavg.items() if k not in not_detect)
    cfg = {"workload": f"{wl['desc']}, {B} frames per SNR", "detector": det, "frames_per_step": frames_per_step,
           "snr_db": snrs}
    if det in ("learned", "learned_hybrid"):
        cfg.update({"k_max": k_max, "margin": margin, "beta": beta, "fallback_K": K})
    if det == "kbest":
        cfg["K"] = K
    if det in ("hybrid", "learned_hybrid"):
        cfg.update({"workers": args.workers, "k_worker": args.k_worker})
    out = {
        "metric": wl["metric"], "value": round(fps, 1), "unit": "frames/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic", "config": cfg,
        "roofline": roofline,
        "errors": {"symbol_errors": counts[:, 1].tolist(), "bit_errors": counts[:, 0].tolist(),
                   "frames_in_error": counts[:, 2].tolist(), "symbols_per_snr": B * M},
        "detect_only_frames_per_s": round(frames_per_step / (det_ms * 1e-3), 1),
        "kernel_avg_ms": {k: round(v, 4) for k, v in kavg.items()},
        "setup_s": round(t_gen, 1),
    }
    kroof = {}
    if det == "learned":
        out["learned"] = {"mean_k_t": round(extra["mean_k_t"], 3),
                          "fallback_fraction": round(extra["fallback_fraction"], 5)}
        # the scheduled K-best expands ~3 survivors a level: its bound is the
        # HBM roof (R read once per frame); its FP32 figure is reported beside it
        kroof["learned"] = dict(hbm_roofline(kbest_bytes_per_frame(n, M, sched=True) * NB, kavg["kbest"]),
                                alu=alu_roofline(kbest_flops_from_counts(sched_counts(extra["ks"], P), P),
                                                 kavg["kbest"]))
    elif det == "kbest":
        kroof["plain"] = alu_roofline(kbest_flops_from_counts(plain_counts(n, P, K) * NB, P), kavg["kbest"])
    if not args.no_graph:
        from paper_2002_09561_amd.graph import CapturedStep

        g = CapturedStep(lambda: (o["counts"].zero_(), step(det, False)))
        for _ in range(args.warmup):  # untimed replays, as the eager steps' warmup
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        gdt = time.perf_counter() - t0
        out["graph_frames_per_s"] = round(frames_per_step * args.steps / gdt, 1)
        out["graph_ms_per_step"] = round(gdt / args.steps * 1e3, 3)
        del g

    # ---------------- comparison legs on the same frames
    names = {"kbest": ("plain_kbest", f"K-best K={K}"),
             "hybrid": ("paper_hybrid", f"SD-K-best, {args.workers} workers x {args.k_worker} survivors"),
             "learned_hybrid": ("learned_hybrid", f"SD-K-best, {args.workers} workers, learned per-level "
                                                  f"survivor counts (capped at {args.k_worker}), node budget "
                                                  f"{args.hybrid_budget or 'none'}, plain K-best K={K} fallback")}
    if not args.no_compare:
        for other in wl["legs"]:
            if other == det or (other == "learned_hybrid" and w is None):
                continue
            odt, oc, okavg, oextra = run(other, True)
            det_ms_o = sum(v for k, v in okavg.items() if k not in not_detect)
            if other == "kbest":
                kroof["plain"] = alu_roofline(kbest_flops_from_counts(plain_counts(n, P, K) * NB, P), okavg["kbest"])
            key, label = names[other]
            out[key] = {"detector": label, "frames_per_s": round(frames_per_step * args.steps / odt, 1),
                        "detect_only_frames_per_s": round(frames_per_step / (det_ms_o * 1e-3), 1),
                        "symbol_errors": oc[:, 1].tolist(), "bit_errors": oc[:, 0].tolist(),
                        "kernel_avg_ms": {k: round(v, 4) for k, v in okavg.items()}}
            if "mean_k_t" in oextra:
                out[key]["mean_k_t"] = round(oextra["mean_k_t"], 3)
                out[key]["fallback_fraction"] = round(oextra["fallback_fraction"], 5)
            if "budget_exhausted_fraction" in oextra:
                out[key]["node_budget"] = args.hybrid_budget
                out[key]["budget_exhausted_fraction"] = round(oextra["budget_exhausted_fraction"], 6)
    if kroof:
        out["kbest_roofline"] = kroof
    # ---------------- ablation: the learned detector's fallback with a constant K
    if not args.no_compare and det == "learned":
        fixed_k = args.fixed_k or max(1, int(round(extra["mean_k_t"])))
        fdt, fc, fkavg, fextra = run("fixed", True)
        fps_fixed = frames_per_step * args.steps / fdt
        out["ablation_fixed_k"] = {
            "detector": f"K-best K={fixed_k} (no network) + the same K={K} fallback",
            "frames_per_s": round(fps_fixed, 1), "symbol_errors": fc[:, 1].tolist(),
            "fallback_fraction": round(fextra["fallback_fraction"], 5),
            "kernel_avg_ms": {k: round(v, 4) for k, v in fkavg.items()},
            "learned_over_ablation": round(fps / fps_fixed, 4)}
    # ---------------- the paper's other detectors on the same frames: linear
    # baselines (Sec. III-A) and K-best over complex levels (its figures' tree)
    if not args.no_compare and args.workload == "c5":
        qr_plain = lambda: mimo.qr_preprocess(H, Y, out=(o["R"], o["z"], None))
        qr_mmse = lambda: mimo.qr_preprocess_mmse(H, Y, SIG2, out=(o["R"], o["z"]))
        legs = {
            "zf": (qr_plain, lambda: mimo.linear_detect(o["R"], o["z"], M, P)),
            "mmse": (qr_mmse, lambda: mimo.linear_detect(o["R"], o["z"], M, P)),
            "mmse_sic": (qr_mmse, lambda: mimo.kbest_detect(o["R"], o["z"], M, P, 1)[0]),
            "mrc": (None, lambda: mimo.mrc_detect(H, Y, P)),
            "complex_kbest_K10": (qr_plain, lambda: mimo.kbest_detect_complex(o["R"], o["z"], M, P, 10)[0]),
        }
        base = {}
        for name, (pre, det_fn) in legs.items():
            if pre:
                pre()
            det_fn()
            ea, eb, ec = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            ea.record(stream)
            if pre:
                pre()
            eb.record(stream)
            s_hat = det_fn()
            ec.record(stream)
            torch.cuda.synchronize()
            err = (s_hat != S_true).view(len(snrs), B, M).sum(dim=(1, 2)).cpu().numpy()
            base[name] = {"frames_per_s": round(frames_per_step / (ea.elapsed_time(ec) * 1e-3), 1),
                          "detect_only_frames_per_s": round(frames_per_step / (eb.elapsed_time(ec) * 1e-3), 1),
                          "symbol_errors": [int(e) for e in err]}
        out["baselines"] = base
    # ---------------- maximum-likelihood reference and matched-BER statistics (untimed)
    if not args.no_ml:
        mimo.qr_preprocess(H, Y, out=(o["R"], o["z"], None))
        ea, eb, ec = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        ea.record(stream)
        sk, pk, _ = mimo.kbest_detect(o["R"], o["z"], M, P, 64)
        r2 = (pk * (1.0 + 1e-4)).contiguous()
        eb.record(stream)
        sm, pm, fm = mimo.sd_hybrid_detect(o["R"], o["z"], M, P, 0, 1, radius2=r2, node_budget=400000)
        ec.record(stream)
        torch.cuda.synchronize()
        sd_ms, warm_ms = eb.elapsed_time(ec), ea.elapsed_time(eb)
        cert1 = float((((fm & mimo.FLAG_CERTIFIED) != 0) & ((fm & mimo.FLAG_FOUND) != 0)).float().mean())
        n_redo = int(((fm & mimo.FLAG_BUDGET_EXHAUSTED) != 0).sum())
        # frames the node budget left unfinished: searched again from their best
        # leaf with their tree spread over a workgroup's wavefronts
        ed = torch.cuda.Event(enable_timing=True)
        mimo.sd_parallel_detect(o["R"], o["z"], M, P, node_budget=20_000_000, redo=True, out=(sm, pm, fm))
        ed.record(stream)
        torch.cuda.synchronize()
        redo_ms = ec.elapsed_time(ed)
        # the same exact SD with every frame's tree spread over a workgroup, for its throughput
        ee, ef = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ee.record(stream)
        sq, _, fq = mimo.sd_parallel_detect(o["R"], o["z"], M, P, radius2=r2, node_budget=20_000_000)
        ef.record(stream)
        torch.cuda.synchronize()
        par_ms = ee.elapsed_time(ef)
        par_cert = ((fq & mimo.FLAG_CERTIFIED) != 0) & ((fq & mimo.FLAG_FOUND) != 0)
        gcert = ((fm & mimo.FLAG_CERTIFIED) != 0) & ((fm & mimo.FLAG_FOUND) != 0)
        sm = torch.where(gcert[:, None], sm, sk)
        ml = sm.cpu().numpy()
        truth = S_true.cpu().numpy()
        # frames the oracle certifies: every frame where the GPU's reference
        # is uncertified or wrong, or where a detector is wrong or disagrees
        # with it, plus a random sample per SNR point
        flag = ~gcert.cpu().numpy() | np.any(ml != truth, axis=1)
        for s in syms.values():
            s = s.cpu().numpy()
            flag |= np.any(s != truth, axis=1) | np.any(s != ml, axis=1)
        rng = np.random.default_rng(args.seed)
        for i in range(len(snrs)):
            flag[i * B + rng.choice(B, size=min(B, args.certify_sample), replace=False)] = True
        idx = np.nonzero(flag)[0]
        t_c = time.perf_counter()
        s_orc, c_orc, Hc, yc = certify_ml(idx, frames, B, P, QAM)
        t_c = time.perf_counter() - t_c
        import oracle

        # the GPU's exact SD against the oracle's on the frames both certified:
        # a difference may only be two points tied for ML (FP64 metrics within
        # 1e-5).  Frames the GPU left uncertified (node budget) keep the K-best
        # result and take the oracle's point as reference.
        both = gcert.cpu().numpy()[idx] & c_orc
        diff = np.any(ml[idx] != s_orc, axis=1) & both
        ties = 0
        if diff.any():
            mg = oracle.metric(Hc[diff], yc[diff], ml[idx][diff], QAM)
            mo = oracle.metric(Hc[diff], yc[diff], s_orc[diff], QAM)
            ties = int(np.sum(np.abs(mg - mo) <= 1e-5 * mo))
        ref = ml.copy()
        ref[idx[c_orc]] = s_orc[c_orc]  # the oracle's point wherever it certified one
        ref_wrong = np.any(ref != truth, axis=1)
        stats = {}
        for name, s in syms.items():
            if name == "fixed":
                continue
            s = s.cpu().numpy()
            wrong = np.any(s != truth, axis=1)
            per = []
            for i in range(len(snrs)):
                sl = slice(i * B, (i + 1) * B)
                x_only = int(np.sum(wrong[sl] & ~ref_wrong[sl]))
                ml_only = int(np.sum(ref_wrong[sl] & ~wrong[sl]))
                both = int(np.sum(wrong[sl] & ref_wrong[sl]))
                dis = int(np.sum(np.any(s[sl] != ref[sl], axis=1)))
                per.append({"snr_db": snrs[i], "symbol_errors": int(np.sum(s[sl] != truth[sl])),
                            "ml_symbol_errors": int(np.sum(ref[sl] != truth[sl])),
                            "frames_wrong": int(wrong[sl].sum()), "ml_frames_wrong": int(ref_wrong[sl].sum()),
                            "detector_only": x_only, "ml_only": ml_only, "both": both,
                            "frame_error_rate_ci95": clopper_pearson(int(wrong[sl].sum()), B),
                            "ml_frame_error_rate_ci95": clopper_pearson(int(ref_wrong[sl].sum()), B),
                            "disagreement_with_ml": dis, "disagreement_rate_ci95": clopper_pearson(dis, B)})
            stats[name] = {"matched": all(p["detector_only"] == 0 for p in per), "per_snr": per}
        sq = sq.cpu().numpy()
        pc = par_cert.cpu().numpy() & gcert.cpu().numpy()
        par_diff = np.nonzero(np.any(sq != ml, axis=1) & pc)[0]
        par_ties = 0
        if par_diff.size:  # both exact: a difference may only be an ML tie
            Hd = np.stack([frames[i // B].H[i % B] for i in par_diff])
            yd = np.stack([frames[i // B].y[i % B] for i in par_diff])
            mg = oracle.metric(Hd, yd, sq[par_diff], QAM)
            mo = oracle.metric(Hd, yd, ml[par_diff], QAM)
            par_ties = int(np.sum(np.abs(mg - mo) <= 1e-5 * mo))
        out["ml_reference"] = {
            "method": "exact Best-FS SD (hybrid kernel, no workers) warm-started by K-best K=64, node budget 4e5; "
                      "the frames it leaves unfinished searched again from their best leaf by the exact SD with the "
                      "tree spread over a workgroup's wavefronts (node budget 2e7); certified by the FP64 oracle "
                      "(K-best K=64 warm radius + Best-FS SD) on every frame any detector gets wrong or disagrees "
                      "on, and on a random sample",
            "symbol_errors": [int(np.sum(ref[i * B:(i + 1) * B] != truth[i * B:(i + 1) * B])) for i in range(len(snrs))],
            "gpu_certified_fraction_budget_4e5": round(cert1, 5),
            "unfinished_frames_searched_again": n_redo, "redo_ms": round(redo_ms, 3),
            "gpu_certified_fraction": round(float(gcert.float().mean()), 5),
            "parallel_sd": {"detect_only_frames_per_s": round(frames_per_step / ((par_ms + warm_ms) * 1e-3), 1),
                            "sd_ms": round(par_ms, 3),
                            "certified_fraction": round(float(par_cert.float().mean()), 5),
                            "differences_from_reference": int(par_diff.size), "of_which_ml_ties": par_ties},
            "oracle_certified_frames": int(c_orc.sum()), "oracle_checked_frames": int(len(idx)),
            "gpu_uncertified_frames_replaced": int(np.sum(~gcert.cpu().numpy()[idx] & c_orc)),
            "both_certified_differences": int(diff.sum()), "of_which_ml_ties": ties,
            "oracle_seconds": round(t_c, 1), "sd_ms": round(sd_ms, 3), "warm_start_ms": round(warm_ms, 3),
            "detect_only_frames_per_s": round(frames_per_step / ((sd_ms + warm_ms) * 1e-3), 1)}
        out["matched_ber"] = {
            "rule": "paired per frame against the oracle-certified ML reference; matched iff no frame is wrong for "
                    "the detector and right for ML at any SNR (allowance 0); Clopper-Pearson 95% intervals",
            "detectors": stats}
        out["matched_ber_headline"] = bool(stats.get(det, {}).get("matched", False))
    if args.copy_probe_mib:
        nbytes = args.copy_probe_mib << 20
        a = torch.empty(nbytes // 4, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
    if not args.no_cpu_baseline:
        legs = [l for l in ("kbest", "hybrid") if l != det and (l in wl["legs"] or l == "kbest")]
        out["cpu_baseline"] = cpu_baseline(frames, w, det if det in ("learned", "kbest") else "kbest", K, meta_run,
                                           args.cpu_baseline_seconds, legs, args.workers, args.k_worker)
    return out


if __name__ == "__main__":
    main()

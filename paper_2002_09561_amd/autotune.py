"""Autotuner for uneven batches: survivors K per (antennas, QAM) class and
the persistent grids of the QR and K-best launches, measured on the GPU.

K per class: the smallest K on a ladder whose symbol errors stay within 5%
of the largest K allowed for that class (K * P <= 256, K <= 64), on
calibration frames spread over the workload's SNR range.  Grids: the fastest
of a few workgroup counts per compute unit for each persistent launch, timed
on a sample uneven batch.  Results are cached as JSON per GPU architecture.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import mimo, uneven
from .framegen import gen_frames, gen_uneven

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE_DIR = os.path.join(HERE, "tuning")


def arch() -> str:
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", "unknown").split(":")[0]


def cache_path(a: str | None = None) -> str:
    return os.path.join(CACHE_DIR, f"uneven_{a or arch()}.json")


def load(a: str | None = None) -> dict | None:
    p = cache_path(a)
    return json.load(open(p)) if os.path.exists(p) else None


def tune_k(antennas=(10, 16, 32, 64), qams=(4, 16, 64), snrs=(8, 12, 16, 20, 24), frames=300,
           ladder=(2, 4, 8, 16, 32, 64), seed=31, log=print):
    table, detail = {}, {}
    for M in antennas:
        for q in qams:
            P = math.isqrt(q)
            ks = [k for k in ladder if k * P <= 256 and k <= 64]
            errs = {k: 0 for k in ks}
            for si, snr in enumerate(snrs):
                f = gen_frames(M, M, q, float(snr), frames, seed=seed, snr_idx=si)
                H = torch.from_numpy(f.H).cuda()
                y = torch.from_numpy(f.y).cuda()
                s = torch.from_numpy(f.s_idx).cuda()
                R, z = mimo.qr_preprocess(H, y)
                for k in ks:
                    sym, _, _ = mimo.kbest_detect(R, z, M, P, k)
                    errs[k] += int((sym != s).sum())
            ref = errs[ks[-1]]
            pick = next(k for k in ks if errs[k] <= 1.05 * ref)
            table[f"{M}x{q}"] = pick
            detail[f"{M}x{q}"] = errs
            log(f"  {M}x{M} {q}-QAM: errors by K {errs} -> K = {pick}")
    return table, detail


def tune_grid(k_table, n_frames=20000, seed=32, qr_mults=(1, 2, 4), kb_mults=(2, 4, 8, 16), log=print):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    fr = gen_uneven(n_frames, seed=seed)
    ub = uneven.UnevenBatch(fr, k_table)

    def t(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(3):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 3

    res = {"qr": {}, "kbest": {}}
    for m in qr_mults:
        res["qr"][m] = t(lambda: mimo.qr_preprocess_uneven(ub.desc, ub.B, ub.max_rx, ub.H, ub.y, ub.R, ub.z,
                                                           ub.counter[0:1], grid=m * cus))
    for m in kb_mults:
        res["kbest"][m] = t(lambda: mimo.kbest_detect_uneven(ub.desc, ub.B, ub.R, ub.z, ub.sym, ub.pd, ub.flags,
                                                             ub.counter[1:2], grid=m * cus))
    qm = min(res["qr"], key=res["qr"].get)
    km = min(res["kbest"], key=res["kbest"].get)
    log(f"  grids (x{cus} CUs): QR {res['qr']} -> {qm}; K-best {res['kbest']} -> {km}")
    return qm * cus, km * cus, res


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--frames", type=int, default=300)
    ap.add_argument("--grid-frames", type=int, default=20000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    mimo.load()
    t0 = time.time()
    table, detail = tune_k(frames=a.frames)
    qg, kg, res = tune_grid(table, n_frames=a.grid_frames)
    out = dict(arch=arch(), k_table=table, errors_by_k=detail, qr_grid=qg, kbest_grid=kg,
               grid_timings_ms={k: {str(m): v for m, v in d.items()} for k, d in res.items()},
               workload="M=N in {10,16,32,64}, QAM in {4,16,64}, SNR uniform 8-24 dB")
    path = a.out or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    json.dump(out, open(path, "w"), indent=1, sort_keys=True)
    print(f"saved {path} ({time.time() - t0:.1f} s)")


if __name__ == "__main__":
    main()

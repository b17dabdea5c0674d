"""The SNR sweep runner on the GPU: a point's counts are those of the same
frames detected directly through the library, and a second run of the same
sweep reads its points back instead of detecting again."""
import math

import pytest
import torch

from paper_2002_09561_amd import mimo, sweep
from paper_2002_09561_amd.framegen import gen_frames

pytestmark = pytest.mark.gpu


def test_sweep_points_and_resume(tmp_path):
    cfg = {"n_rx": 8, "n_tx": 8, "qam": 16, "detector": "kbest", "K": 16, "frames": 1000, "seed": 3}
    path = str(tmp_path / "s.jsonl")
    recs = sweep.run_sweep(cfg, [6.0, 10.0], lambda s: sweep.gpu_point(cfg, s), path, log=lambda *_: None)
    P = math.isqrt(cfg["qam"])
    for rec in recs:
        f = gen_frames(8, 8, 16, rec["snr_db"], 1000, seed=3, snr_idx=sweep.snr_stream(rec["snr_db"]))
        R, z = mimo.qr_preprocess(torch.from_numpy(f.H).cuda(), torch.from_numpy(f.y).cuda())
        sym = mimo.kbest_detect(R, z, 8, P, 16)[0]
        c = mimo.error_count(sym, torch.from_numpy(f.s_idx).cuda(), P).tolist()
        assert [rec["bit_errors"], rec["symbol_errors"], rec["frames_in_error"]] == c
        assert rec["frames"] == 1000 and rec["symbols"] == 8000
    assert recs[0]["symbol_errors"] > recs[1]["symbol_errors"] > 0
    again = sweep.run_sweep(cfg, [10.0, 6.0], lambda s: pytest.fail("point detected again"), path,
                            log=lambda *_: None)
    assert [r["snr_db"] for r in again] == [10.0, 6.0]

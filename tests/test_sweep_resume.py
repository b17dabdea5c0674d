"""Resume logic of the SNR sweep runner (host only: the point function is a
stub, no GPU and no detector)."""
import json

import pytest

from paper_2002_09561_amd import sweep


def _stub(calls, fail_at=None):
    def run_point(snr):
        calls.append(snr)
        if fail_at is not None and snr == fail_at:
            raise RuntimeError("interrupted")
        return {"symbol_errors": int(100 - snr), "frames": 10}
    return run_point


CFG = {"n_rx": 4, "n_tx": 4, "qam": 16, "detector": "kbest", "K": 8, "frames": 10, "seed": 0}


def test_resume_runs_only_missing_points(tmp_path):
    path = str(tmp_path / "s.jsonl")
    calls = []
    with pytest.raises(RuntimeError):
        sweep.run_sweep(CFG, [0, 5, 10, 15], _stub(calls, fail_at=10), path, log=lambda *_: None)
    assert calls == [0.0, 5.0, 10.0]
    # the two finished points are on disk, the interrupted one is not
    assert sorted(sweep.load_done(path, sweep.config_key(CFG))) == [0.0, 5.0]
    calls.clear()
    recs = sweep.run_sweep(CFG, [0, 5, 10, 15], _stub(calls), path, log=lambda *_: None)
    assert calls == [10.0, 15.0]
    assert [r["snr_db"] for r in recs] == [0.0, 5.0, 10.0, 15.0]
    assert [r["symbol_errors"] for r in recs] == [100, 95, 90, 85]
    # a third run finds everything
    calls.clear()
    sweep.run_sweep(CFG, [15, 0], _stub(calls), path, log=lambda *_: None)
    assert calls == []


def test_other_configuration_is_not_reused(tmp_path):
    path = str(tmp_path / "s.jsonl")
    calls = []
    sweep.run_sweep(CFG, [0, 5], _stub(calls), path, log=lambda *_: None)
    other = dict(CFG, K=16)
    calls.clear()
    sweep.run_sweep(other, [0, 5], _stub(calls), path, log=lambda *_: None)
    assert calls == [0.0, 5.0]
    # key order in the configuration does not matter
    calls.clear()
    sweep.run_sweep(dict(reversed(list(CFG.items()))), [0, 5], _stub(calls), path, log=lambda *_: None)
    assert calls == []


def test_line_cut_short_is_ignored_and_point_rerun(tmp_path):
    path = str(tmp_path / "s.jsonl")
    calls = []
    sweep.run_sweep(CFG, [0], _stub(calls), path, log=lambda *_: None)
    key = sweep.config_key(CFG)
    with open(path, "a", encoding="utf-8") as f:  # a crash in the middle of writing the 5 dB point
        f.write(json.dumps({"key": key, "config": CFG, "snr_db": 5.0, "symbol_errors": 95})[:40])
    assert sorted(sweep.load_done(path, key)) == [0.0]
    calls.clear()
    recs = sweep.run_sweep(CFG, [0, 5], _stub(calls), path, log=lambda *_: None)
    assert calls == [5.0]
    assert [r["snr_db"] for r in recs] == [0.0, 5.0]
    # the new record starts a line of its own: every whole line parses
    lines = open(path, encoding="utf-8").read().splitlines()
    parsed = []
    for ln in lines:
        try:
            parsed.append(json.loads(ln))
        except json.JSONDecodeError:
            pass
    assert sorted(r["snr_db"] for r in parsed) == [0.0, 5.0]


def test_snr_stream_tags_are_distinct_and_list_independent():
    tags = {sweep.snr_stream(s) for s in (-5.0, 0.0, 0.1, 4.0, 20.0, 28.0)}
    assert len(tags) == 6 and all(t >= 0 for t in tags)
    assert sweep.snr_stream(20.0) == sweep.snr_stream(20.0000001)

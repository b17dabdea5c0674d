"""bench.py's command-line contract on the host: runs on several GPUs are
refused with a message, and the extra configurations of the default line
report a failure in place of their numbers instead of ending the run."""
import argparse
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_extra_workloads_report_failures(monkeypatch):
    def boom(args):
        raise RuntimeError(f"no device for {args.workload}")

    monkeypatch.setattr(bench, "uneven_run", boom)
    monkeypatch.setattr(bench, "sweep_run", boom)
    sys_argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        args = bench.parse()
    finally:
        sys.argv = sys_argv
    assert isinstance(args, argparse.Namespace) and args.workload == "c5" and not args.no_extra
    res = bench.extra_workloads(args)
    assert set(res) == {"uneven", "c4"}
    assert "no device for uneven" in res["uneven"]["error"]
    assert "no device for c4" in res["c4"]["error"]
    # the caller's arguments are left as they were
    assert args.workload == "c5" and args.no_ml is False

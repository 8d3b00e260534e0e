"""Host-side logic of bench.py (no GPU): the one-GPU guard, the CPU oracle
baseline on small shapes of both spatial paths, and the rule that recorded
HBM traffic is reported only for the kernel choice it was counted with."""
import dataclasses
import json
import math
import os
import subprocess
import sys

import bench
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in out["error"]


def _check_baseline(res, iters, flexible):
    assert res["kind"] == "oracle" and res["unit"] == "solves/s"
    assert math.isfinite(res["value"]) and res["value"] > 0
    assert res["cores"] >= 1
    assert ("flexible" in res["sample"]) == flexible
    assert str(list(iters)) in res["sample"]
    # the composition: k (apply + matvec) dominates; a solve is slower than
    # k applies alone
    k = sum(iters)
    assert 1.0 / res["value"] * len(iters) >= k * res["per_apply_s"]


def test_cpu_baseline_sine_transform_path():
    cfg = dataclasses.replace(W.WORKLOADS["2d-nx31-nt32"], nx=15, nt=16)
    res = bench.cpu_baseline(cfg, [12, 14], budget_s=2.0)
    _check_baseline(res, [12, 14], flexible=False)
    assert "splu" in res["sample"]


def test_cpu_baseline_multigrid_path():
    cfg = dataclasses.replace(W.WORKLOADS["3d-nx63-nt128-vara-mg"], nx=7, nt=8)
    res = bench.cpu_baseline(cfg, [9], budget_s=2.0, flexible=True)
    _check_baseline(res, [9], flexible=True)
    assert "V-cycles" in res["sample"]


def test_recorded_traffic_needs_the_counted_kernel_choice():
    path = os.path.join(ROOT, "profiles", "kernels_2d-nx511-nt512-fp64-and-mixed.md")
    rec = None
    for line in open(path):
        if line.startswith("traffic: "):
            rec = json.loads(line[len("traffic: "):])
    assert rec is not None
    choices = {leg: dict(ch) for leg, ch in rec["kernels"].items()}
    fam = "gs_update"
    got = bench.recorded_traffic(rec["workload"], fam, choices)
    # the record matches its own sources only while the kernels are unchanged;
    # either way a different kernel choice must never be given the record
    if got is not None:
        assert got == rec["families"][fam]["bytes_per_launch"]
    other = {leg: dict(ch, gs_update=3 - ch["gs_update"]) for leg, ch in choices.items()}
    assert bench.recorded_traffic(rec["workload"], fam, other) is None
    assert bench.recorded_traffic("no-such-workload", fam, choices) is None


def test_paper_context_for_every_workload():
    for cid in (1, 2, 3, 4, 5):
        ctx = bench.paper_context(cid)
        json.dumps(ctx)
        assert "M4 Pro" in ctx["setup"] and ctx["rows"]
        for row in ctx["rows"]:
            assert row["iters"] > 0 and row["cpu_s"] > 0 and row["source"].startswith("Table")
    # the workloads the paper has no run of say so
    assert "not reported" in bench.paper_context(3)["note"]

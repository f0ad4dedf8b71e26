"""The benchmark's host-side contract (no GPU): it refuses more than one GPU
with a message, and reports a counter-measured figure only for the kernel
sources it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_measured_figures_follow_the_source_hash(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    # every recorded kernel names a hash of 16 hex digits and positive bytes
    for name, k in rec["kernels"].items():
        assert len(k["source_sha256_16"]) == 16 and k["traffic_bytes"] > 0, name
    # a figure recorded for other sources is not reported
    kern = dict(rec["kernels"]["mcc_fj_generated2"], source_sha256_16="0" * 16)
    fake = dict(rec, kernels={"mcc_fj_generated2": kern})
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(fake))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic(bench.FJ_KERNEL, bench.FJ_SOURCES) is None
    # an unknown kernel or workload size has no figure
    assert bench.measured_traffic("no_such_kernel", bench.FJ_SOURCES) is None
    assert bench.measured_traffic(bench.FJ_KERNEL, bench.FJ_SOURCES, 12345) is None


def test_issue_roofline_only_for_the_measured_configuration():
    assert bench.issue_roofline(0.19, 10001, 32) is None
    assert bench.solver_counter("traffic_bytes", 10000, 48) is None

"""bench.py pieces that run without a GPU: the one-GPU refusal, the counter
summary lookup (keyed on workload and on a hash of the solve sources) and the
CPU baseline record."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_lookup_follows_workload_and_sources(monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        text = fh.read()
    recorded = [ln.split("`")[1] for ln in text.splitlines() if ln.startswith("- source_hash:")][0]
    monkeypatch.setattr(bench, "solve_source_hash", lambda: recorded)
    v = bench.measured_traffic(4)
    assert v is not None and v > 1e11
    assert bench.measured_traffic(2) is None          # another workload
    monkeypatch.setattr(bench, "solve_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic(4) is None          # sources changed since counting


def test_nij_traffic_lookup_follows_its_sources():
    with open(bench.TRAFFIC_NIJ_FILE) as fh:
        text = fh.read()
    recorded = [ln.split("`")[1] for ln in text.splitlines() if ln.startswith("- source_hash:")][0]
    assert bench.measured_traffic(4, bench.TRAFFIC_NIJ_FILE, lambda: recorded) > 1e11
    assert bench.measured_traffic(4, bench.TRAFFIC_NIJ_FILE, lambda: "0" * 16) is None


def test_cpu_baseline_record():
    from paper_2106_06149_amd import synth
    s = synth.workload(1)
    rec = bench.cpu_baseline(s, 6, workers=2)
    assert rec["kind"] == "oracle" and rec["unit"] == "pair-blocks/s"
    assert rec["value"] > 0 and rec["cores"] == 2
    assert rec["sample"].startswith("6 seeded clusters") and "2 worker processes" in rec["sample"]
    assert rec["cpu_model"] and rec["cpu_count"] >= 1

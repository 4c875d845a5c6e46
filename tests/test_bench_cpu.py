"""The measurement script's host-side contract (CPU only): the one-GPU refusal,
the workload list, the traffic figure's tie to the kernel sources it was
measured on, and the CPU baseline record."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr
    assert r.stdout.strip() == ""   # no JSON line


def test_workloads_listed():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("single", "batch", "serve", "precision", "sliding", "postproc", "frames132", "copycal"):
        assert w in r.stdout


def test_traffic_follows_the_kernel_sources(tmp_path, monkeypatch):
    sha = bench.kernel_source_sha()
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"source_sha": sha, "bytes_per_launch": 123.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic() == 123.0
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"source_sha": "0" * 16, "bytes_per_launch": 123.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() is None


def test_committed_traffic_summary_is_well_formed():
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    for key in ("source_sha", "bytes_per_launch", "fetch_bytes", "write_bytes",
                "algorithmic_bytes", "fetch_factor", "write_factor", "commands"):
        assert key in t
    assert t["bytes_per_launch"] == t["fetch_bytes"] + t["write_bytes"]
    # the pass re-reads nothing: measured traffic within a few percent above
    # the 5 words per entry of the algorithm
    assert 1.0 <= t["bytes_per_launch"] / t["algorithmic_bytes"] <= 1.05


def test_cpu_baseline_record():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((300, 6))
    rec = bench.cpu_baseline(X, 1.0 / np.sqrt(300), budget_s=0.2, max_iters=3, one_thread_iters=2)
    assert rec["kind"] == "oracle" and rec["unit"] == "pixel-frames/s per ALM iter"
    assert rec["value"] > 0 and rec["cores"] >= 1 and rec["s_per_iter"] > 0
    assert "300x6" in rec["sample"]
    assert rec["one_thread"]["iters"] == 2 and rec["one_thread"]["value"] > 0

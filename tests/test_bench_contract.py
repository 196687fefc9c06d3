"""Host-side parts of the benchmark's contract (no device needed).

* More than one GPU is refused with a message and a non-zero exit before any
  work: every measured figure here is one GPU's.
* The traffic figure is tied to the kernel sources it was counted on: the
  committed summary names a source hash and per-kernel counts, and a hash
  that differs turns the figure off instead of reporting stale bytes.
"""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_figure_follows_the_source_hash(monkeypatch):
    import bench
    with open(bench.TRAFFIC_FILE) as fh:
        line = next(l for l in fh if l.startswith("traffic-json:"))
    t = json.loads(line.split(":", 1)[1])
    assert {"source_sha256", "fetch_factor", "write_factor", "kernels"} <= set(t)
    name = sorted(t["kernels"])[0]
    k = t["kernels"][name]
    want = 1024.0 * (k["fetch_kib"] * t["fetch_factor"] + k["write_kib"] * t["write_factor"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: t["source_sha256"])
    assert bench.traffic_bytes(name) == pytest.approx(want)
    assert bench.traffic_bytes("no_such_kernel") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.traffic_bytes(name) is None

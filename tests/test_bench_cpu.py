"""Host logic of bench.py (no GPU): the one-GPU contract, the harmonic number
behind the points model, and the use of the committed HBM counter summary
(reported only for the kernel sources, workload size and variant it was taken
on)."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_harmonic():
    assert bench.harmonic(1) == 1.0
    assert abs(bench.harmonic(1024) - (np.log(1024) + 0.5772156649 + 1 / 2048)) < 1e-6


def test_measured_traffic_follows_the_record(tmp_path, monkeypatch):
    rec = {"kernel_source_sha256": bench.kernel_source_sha(), "num_sets": 10,
           "calibration": {"fetch_factor": 2.0, "write_factor": 1.0},
           "kernels": {"pmh1": {"fetch_kib": 3.0, "write_kib": 5.0}}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    v, note = bench.measured_traffic(1, 10)
    assert v == 3.0 * 1024 * 2.0 + 5.0 * 1024 * 1.0 and "FETCH_SIZE" in note
    assert bench.measured_traffic(3, 10)[0] is None       # no counters for the variant
    assert bench.measured_traffic(1, 11)[0] is None       # another workload size
    rec["kernel_source_sha256"] = "0" * 64
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(1, 10)[0] is None       # kernel changed since
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic(1, 10)[0] is None


@pytest.mark.parametrize("variant", [1, 3])
def test_committed_record_is_complete(variant):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    k = rec["kernels"][f"pmh{variant}"]
    assert k["fetch_kib"] > 0 and k["write_kib"] > 0
    assert rec["calibration"]["fetch_factor"] > 0 and rec["calibration"]["write_factor"] > 0
    assert rec["num_sets"] == 100_000


def test_profiled_runs_can_skip_the_autotuner(monkeypatch):
    """Profiled skewed-batch runs pass --no-autotune, so their kernel traces hold
    only default-tuning launches; the plain bench keeps the autotuned leg."""
    monkeypatch.setattr(sys, "argv", ["bench.py", "--no-autotune"])
    assert bench.parse().no_autotune
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    assert not bench.parse().no_autotune

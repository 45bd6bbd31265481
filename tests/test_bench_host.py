"""Host logic of bench.py (no GPU): the one-GPU contract and the traffic record lookup."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


@pytest.fixture
def fake_record(tmp_path, monkeypatch):
    src = tmp_path / "sweep2d.hip"
    src.write_text("// kernel source\n")
    rec = {"sweep_source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "fetch_bytes_per_launch": 1000.0, "write_bytes_per_launch": 3000.0,
           "copy_fetch_factor": 0.5, "copy_write_factor": 1.0}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(bench, "SWEEP_SOURCE", str(src))
    return src


def test_traffic_scaled_by_copy_calibration(fake_record):
    # fetch 1000 B read at half the copy's rate -> 2000 B; writes unscaled -> 3000 B
    assert bench.measured_traffic() == pytest.approx(5000.0)


def test_traffic_null_once_the_kernel_source_changed(fake_record):
    fake_record.write_text("// kernel source, edited after profiling\n")
    assert bench.measured_traffic() is None


def test_traffic_null_without_a_record(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() is None

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
    src = tmp_path / "sweep3d.hip"
    src.write_text("// kernel source\n")
    rec = {"sweep_source_sha256": hashlib.sha256(src.read_bytes()).hexdigest(),
           "fetch_bytes_per_launch": 1000.0, "write_bytes_per_launch": 3000.0,
           "copy_fetch_factor": 0.5, "copy_write_factor": 1.0}
    (tmp_path / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    monkeypatch.setattr(bench, "CSRC", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC", {5: ("traffic.json", "sweep3d.hip")})
    return src


def test_traffic_scaled_by_copy_calibration(fake_record):
    # fetch 1000 B read at half the copy's rate -> 2000 B; writes unscaled -> 3000 B
    assert bench.measured_traffic(5) == pytest.approx(5000.0)


def test_traffic_null_once_the_kernel_source_changed(fake_record):
    fake_record.write_text("// kernel source, edited after profiling\n")
    assert bench.measured_traffic(5) is None


def test_traffic_null_without_a_record(monkeypatch, tmp_path):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.measured_traffic(5) is None


def test_algorithmic_bytes_match_the_per_update_figures():
    """O p [2 + n_rhs (n_P + n_out)] per cell and launch, divided by the updates of the
    launch: 9.6 B (256^2 S8 FP64 RLMDG, one source) and 7.7 B (128^3 3D S8 FP32 RLMDG,
    eight sources) per cell-direction update."""
    b2 = bench.sweep_bytes_per_launch(65536, "rlmdg", 2, 1, 8) / (65536 * 40)
    b5 = bench.sweep_bytes_per_launch(128 ** 3, "rlmdg", 3, 8, 4) / (128 ** 3 * 80 * 8)
    assert b2 == pytest.approx(9.6)
    assert b5 == pytest.approx(7.7)

"""Host-side arithmetic of bench.py: the algorithmic bytes behind every roofline figure, the
minimum bytes of a blocked pass, the traffic record lookup and the single-GPU refusal."""
import json
import subprocess
import sys

import pytest

import bench


def test_algorithmic_bytes_of_the_configurations():
    # config 2: 3 vector streams of 262144 sites x 32 complex64 values, plus 3 forward bonds per site
    assert bench.algorithmic_bytes_per_step(64 ** 3, 32, True, 4, False, 3) == 207_618_048
    # config 4: 3 streams of 2048^2 x 64 FP32 values plus the FP32 diagonal
    assert bench.algorithmic_bytes_per_step(2048 ** 2, 64, False, 4, True, 0) == 3 * 2 ** 30 + 4 * 2048 ** 2
    # one site-moment-vector update costs 1.5 e bytes of vectors (two moments per step)
    N, R = 1000, 8
    assert bench.algorithmic_bytes_per_step(N, R, False, 4, False, 0) / (N * 2 * R) == 1.5 * 4


def test_blocked_pass_minimum_bytes():
    # four vector transfers per pass of D steps plus the diagonal once per step
    assert bench.tb_pass_bytes(2048 ** 2, 64, False, 4, True, 4) == 4 * 2 ** 30 + 4 * 16 * 2 ** 20
    assert bench.tb_pass_bytes(100, 4, True, 8, False, 3, bonds_per_site=2) == 4 * 100 * 4 * 16 + 3 * 100 * 2 * 2 * 8


def test_chunk_group_and_depth_rules():
    assert bench.tb_groups(16, 2048) == 1          # a 32-site window already
    assert bench.tb_groups(32, 2048) == 4          # groups of 8 chunks: 64-site windows
    assert bench.tb_groups(128, 40) == 8           # groups of 16 chunks: a 32-site window within L_x = 40
    assert bench.tb_groups(32, 2048, group=0) == 1
    assert bench.tb_depth(-1, 1, 16) == 4          # FP32 real hopping
    assert bench.tb_depth(-1, 0, 16) == 3          # FP64
    assert bench.tb_depth(-1, 1, 16, spin=True) == 3
    assert bench.tb_depth(-1, 1, 32, spin=True, Lx=2048) == 4   # spin hopping in chunk groups
    assert bench.tb_depth(-1, 0, 32, spin=True, Lx=2048) == 3
    assert bench.tb_depth(6, 1, 64, Lx=8) == 2     # capped at a quarter of a 8-site window


def test_traffic_record_is_keyed_by_kernel_and_source_digest(tmp_path, monkeypatch):
    rec = {"config4": {"kernel": "k", "source_digest": bench.kernel_source_digest(), "traffic_bytes_per_step": 5.0}}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(path))
    assert bench.measured_traffic("config4", "k") == 5.0
    assert bench.measured_traffic("config4", "other kernel") is None
    assert bench.measured_traffic("config2", "k") is None
    rec["config4"]["source_digest"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("config4", "k") is None


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "error" in json.loads(out.stdout.strip().splitlines()[-1])

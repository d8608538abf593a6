"""bench.py's host logic (CPU only): the one-GPU refusal, the algorithmic
bytes per cell behind the roofline, and the rule that a committed HBM traffic
figure is reported only while the stage-kernel sources it was measured on are
unchanged."""
import os
import subprocess
import sys

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


def test_algorithmic_bytes_per_cell():
    # stage 1: Q^s 40 + metrics 80 + write 40; stages 2-3 add Q^n 40; mean over 3 stages
    assert bench.stage_bytes_per_cell(False) == pytest.approx((160 + 2 * 200) / 3)
    assert bench.stage_bytes_per_cell(True) == pytest.approx((160 + 2 * 200) / 3 + 8)


def test_traffic_needs_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_sha", lambda sources=None: "abc123")
    assert bench.read_traffic("stage_x") is None                       # no summary
    (prof / "stage_x_pmc.txt").write_text("# comment: ignored\nsource_sha: abc123\nhbm_bytes_per_launch: 12345\n")
    assert bench.read_traffic("stage_x") == 12345.0
    (prof / "stage_x_pmc.txt").write_text("source_sha: 0000\nhbm_bytes_per_launch: 12345\n")
    assert bench.read_traffic("stage_x") is None                       # kernels changed since


def test_source_sha_covers_the_stage_kernel_sources():
    sha = bench.source_sha()
    assert len(sha) == 16 and int(sha, 16) >= 0

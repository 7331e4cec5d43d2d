"""Host-side checks of the benchmark script's contract (no GPU)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("good_hash,launch,expect", [
    (True, "N=65536 T=2000 fp32", 123456.0),
    (False, "N=65536 T=2000 fp32", None),
    (True, "N=1024 T=2000 fp32", None),
])
def test_traffic_record_applies_only_to_its_sources_and_launch(tmp_path, monkeypatch, good_hash, launch, expect):
    sha = bench.kernel_sources_sha256() if good_hash else "0" * 64
    rec = tmp_path / "traffic.md"
    rec.write_text("# title\n\n| a | b |\n|---|---|\n\n"
                   f"source_sha256: {sha}\nlaunch: {launch}\nhbm_bytes_per_launch: 123456\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(rec))
    assert bench._measured_traffic(65536, 2000, "fp32") == expect


def test_missing_traffic_record_gives_null(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "absent.md"))
    assert bench._measured_traffic(65536, 2000, "fp32") is None

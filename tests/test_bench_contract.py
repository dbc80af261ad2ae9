"""Host-side checks of bench.py's contract (no GPU): it refuses more than one
GPU with a message, and the roofline's traffic figure is taken from a counter
summary only while that summary's recorded source digest matches the
library sources."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_is_read_only_for_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_digest", lambda: "c0ffee")
    val, note = bench.profiled_traffic("w", "fp64")
    assert val is None and "no counter summary" in note
    (prof / "k_gemm_w_fp64.md").write_text(
        "text\ntraffic_bytes_per_launch: 1.5e+09\nsources_sha256: c0ffee\n")
    val, note = bench.profiled_traffic("w", "fp64")
    assert val == pytest.approx(1.5e9)
    (prof / "k_gemm_w_fp64.md").write_text("traffic_bytes_per_launch: 1.5e+09\nsources_sha256: 00\n")
    val, note = bench.profiled_traffic("w", "fp64")
    assert val is None and "other sources" in note

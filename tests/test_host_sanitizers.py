"""The host-side nested-dissection analysis built with AddressSanitizer and
UndefinedBehaviorSanitizer (g++, host code only) and run over grids that
exercise the channel-row and band-edge cuts, small leaves and chained
separators (tests/sanitize_analyze.cpp checks the structure it builds)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_analysis_is_clean_under_address_and_ub_sanitizers(tmp_path):
    exe = tmp_path / "sanitize_analyze"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "sanitize_analyze.cpp"),
           os.path.join(ROOT, "paper_2306_09257_amd", "csrc", "analyze.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "FAIL" not in r.stdout and "runtime error" not in r.stderr

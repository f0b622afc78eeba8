"""Host logic of the serving scheduler (no GPU): the device-memory arena's
first-fit placement and coalescing, the skip-ahead admission pass, and a
randomized comparison with a granule-bitmap model.  The checks are a small
C++ program built with g++ against the scheduler's own header."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_arena_and_admission(tmp_path):
    exe = tmp_path / "arena_check"
    src = os.path.join(ROOT, "tests", "native", "arena_check.cpp")
    inc = os.path.join(ROOT, "paper_0906_5170_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-I", inc, src,
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert "arena ok" in out.stdout

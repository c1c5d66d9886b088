"""The server's device-budget allocator (csrc/pool.h, pure host C++) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run against
a byte-occupancy model (tests/native/pool_check.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2005_06727_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_region_pool_against_model(tmp_path):
    exe = str(tmp_path / "pool_check")
    src = os.path.join(ROOT, "tests", "native", "pool_check.cpp")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, src, "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "0 failures" in r.stdout

"""The aggregation region (paper Section V-D) on a fake executor with real
threads: team formation (idle executor, full team behind a busy one),
chunked buffers, operations run once per team by its last member, team
failure on a mismatched call or an arena overflow.  Built with g++ and
AddressSanitizer/UBSan (host code only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_aggregation_region(tmp_path):
    exe = tmp_path / "region_core_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", os.path.join(HERE, "region_core_test.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all region checks passed" in r.stdout

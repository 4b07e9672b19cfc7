"""The aggregation policy (when held sub-grid tasks are launched as one
batch) on a fake executor with a virtual clock: width, idle-stream, timeout,
byte-budget and parameter-change rules, ticket/result mapping, error paths.
Built with g++ and AddressSanitizer/UBSan (host code only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_aggregation_policy(tmp_path):
    exe = tmp_path / "agg_policy_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-omit-frame-pointer", os.path.join(HERE, "agg_policy_test.cpp"),
                    "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all policy checks passed" in r.stdout

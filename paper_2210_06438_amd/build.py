"""Compile libhydroagg.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhydroagg.so")
SOURCES = [os.path.join(HERE, "csrc", "hydro_api.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay disabled in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    deps = SOURCES + glob.glob(os.path.join(HERE, "csrc", "*.hpp")) + \
        [os.path.join(os.path.dirname(HERE), "include", "hydroagg.h")]
    for d in deps:
        if not os.path.exists(d):
            raise FileNotFoundError(d)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

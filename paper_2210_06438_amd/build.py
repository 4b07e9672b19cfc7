"""Compile libhydroagg.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libhydroagg.so")
# every translation unit of the library: csrc/*.hip
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay disabled in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def source_files():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.hpp")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.cpp")) +
                  [os.path.join(os.path.dirname(HERE), "include", "hydroagg.h")])


def source_hash() -> str:
    """Short hash of every source the library is built from; the library
    reports it through hydro_version() so measurements can be tied to the
    exact kernel they were taken on."""
    h = hashlib.sha1()
    for f in source_files():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("hydro_kernel.hpp", "hydro_lds8.hpp", "hydro_q4.hpp",
                            "hydro_mixed.hpp", "hydro_pattern.hpp", "hydro_step26.hpp")]


def kernel_hash() -> str:
    """Short hash of what fixes the hydro kernels' machine code: their
    sources (device code and launch geometry) and the compile flags.  Host
    code around them can change without changing it, so a kernel measurement
    (profiler counters) stays tied to the kernels it was taken on."""
    h = hashlib.sha1(" ".join(FLAGS).encode())
    for f in KERNEL_SOURCES:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def build(verbose: bool = False) -> str:
    for d in SOURCES:
        if not os.path.exists(d):
            raise FileNotFoundError(d)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, f'-DHYDRO_SRC_HASH="{source_hash()}"',
           f'-DHYDRO_KERNEL_HASH="{kernel_hash()}"', *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Builds libsco.so (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsco.so")
SOURCES = [os.path.join(CSRC, "sco_kernels.hip"), os.path.join(CSRC, "sco_api.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # decisions shared with the CPU reference are evaluated exactly as written
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


DRIVER = os.path.join(HERE, "sco_drive")
DRIVER_SRC = os.path.join(CSRC, "sco_drive.cpp")


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, *FLAGS, "-o", tmp, *SOURCES])
    os.replace(tmp, LIB)
    # native C-ABI driver (profiling, usage example), linked against the library
    tmp = DRIVER + ".tmp"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-Wall", "-o", tmp, DRIVER_SRC,
                           f"-L{HERE}", "-lsco", f"-Wl,-rpath,{HERE}", "-Wl,-rpath,$ORIGIN"])
    os.replace(tmp, DRIVER)
    return LIB


if __name__ == "__main__":
    print(build())

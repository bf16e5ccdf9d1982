"""Build liborbit_hip.so (hipcc, gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liborbit_hip.so")
SOURCES = ["orbit_lib.hip", "orbit_prep.hip", "orbit_count.hip", "orbit_combine.hip",
           "orbit_common.h", "orbit_tables.h"]


def hipcc_command(out: str = LIB):
    return ["hipcc", "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(HERE, "..", "include"),
            "-o", out, os.path.join(CSRC, "orbit_lib.hip")]


def build() -> str:
    """Compile the HIP library (always recompiles)."""
    tmp = LIB + ".tmp"
    subprocess.check_call(hipcc_command(tmp))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

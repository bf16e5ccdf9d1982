"""Build liborbit_hip.so (hipcc, gfx950) in-tree.

Two builds of the same sources:
* ``liborbit_hip.so`` -- the library;
* ``liborbit_hip_tiles.so`` -- the same code with every LDS tile shrunk
  (clique bit rows, pair-sweep wheel maps, the long triangle-list sort) and
  the per-source maps kept in HBM, so that graphs small enough for the CPU
  oracle take the paths that only hubs and large graphs take in the library
  build.  Only the tests load it.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liborbit_hip.so")
LIB_TILES = os.path.join(HERE, "liborbit_hip_tiles.so")
SOURCES = ["orbit_lib.hip", "orbit_prep.hip", "orbit_count.hip", "orbit_combine.hip",
           "orbit_sched.hip", "orbit_common.h", "orbit_tables.h"]
# tile sizes of the test build (each the smallest its kernel accepts or a
# size a 40..120-vertex graph exceeds; no per-source maps in LDS)
SMALL_TILES = {"CLQ_LDS_D": 16, "PAIR_KMAP_LDS": 16, "TL_SORT_LDS": 128, "LDS_MAP_BUDGET": 0}


def hipcc_command(out: str = LIB, defines=None):
    cmd = ["hipcc", "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(HERE, "..", "include")]
    for k, v in (defines or {}).items():
        cmd.append(f"-D{k}={v}")
    return cmd + ["-o", out, os.path.join(CSRC, "orbit_lib.hip")]


def _build_one(out, defines=None):
    tmp = out + ".tmp"
    subprocess.check_call(hipcc_command(tmp, defines))
    os.replace(tmp, out)
    return out


def build() -> str:
    """Compile both builds (always recompiles); returns the library's path."""
    _build_one(LIB)
    _build_one(LIB_TILES, SMALL_TILES)
    return LIB


if __name__ == "__main__":
    print(build())

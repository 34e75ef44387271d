"""Build step for the HIP library (gfx950) and the CPU oracle.

``build()`` always recompiles ``csrc/*.hip`` into ``libdtw_hip.so`` next to
this file with hipcc.  Packed-FP32 instruction selection is disabled for all
device code.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdtw_hip.so")
SOURCES = ["dtw_wave.hip", "dtw_plan.hip", "dtw_api.hip", "dtw_server.hip", "dtw_edit.hip", "dtw_local.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc_command(out=LIB):
    return ["hipcc", *HIPCC_FLAGS, *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    subprocess.run(hipcc_command(tmp), check=True,
                   stdout=None if verbose else subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

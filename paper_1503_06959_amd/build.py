"""Builds the gfx950 library libkpd.so in-tree with hipcc.

Usage: python -m paper_1503_06959_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkpd.so")
SOURCES = [os.path.join(CSRC, "kpd_api.cpp"), os.path.join(CSRC, "kpd_kernels.hip"), os.path.join(CSRC, "kpd_group.hip"),
           os.path.join(CSRC, "kpd_tcd.cpp"), os.path.join(CSRC, "kpd_tcd.hip"),
           os.path.join(CSRC, "kpd_layers.cpp"), os.path.join(CSRC, "kpd_layers.hip"),
           os.path.join(CSRC, "kpd_noalloc.hip")]
HEADERS = [os.path.join(CSRC, "kpd_geom.h"), os.path.join(CSRC, "kpd_kernels.h"), os.path.join(CSRC, "kpd_tcd.h"), os.path.join(CSRC, "kpd_errors.h"), os.path.join(CSRC, "kpd_group.h"),
           os.path.join(CSRC, "kpd_layers.h"), os.path.join(CSRC, "kpd_fit.h"), os.path.join(CSRC, "kpd_trace.h"),
           os.path.join(os.path.dirname(HERE), "include", "kpd.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # floating expressions as written: no fused multiply-adds
    "-ffp-contract=off",
]


# named ranges around the entry points (roctx)
LIBS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES, *LIBS]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libkpd.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

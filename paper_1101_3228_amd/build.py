"""Build the qtree HIP library (libqtree.so) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqtree.so")
# calibration program of the ALU rooflines (VALU issue rate per opcode)
RATES_SRC = os.path.join(CSRC, "valu_rates.hip")
RATES_BIN = os.path.join(PKG, "valu_rates")

SOURCES = ["api.cpp", "batch.cpp", "quantizer.cpp", "mlp_api.cpp", "fwd.hip", "count.hip",
           "bdp.hip", "diag.hip", "mlp.hip", "swing.hip", "lloyd.hip", "lloyd_api.cpp",
           "strat.hip"]

# -ffp-contract=off: the sample arithmetic is a fixed sequence of IEEE
# operations (explicit fmaf only); packed FP32 instructions are disabled.
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
         "-ffp-contract=off", "-fno-fast-math",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libqtree.so")
    os.replace(tmp, LIB)
    build_rates(verbose)
    return LIB


def build_rates(verbose: bool = False) -> str:
    flags = [f for f in FLAGS if f not in ("-shared", "-fPIC")]
    tmp = RATES_BIN + ".tmp"
    cmd = [hipcc(), *flags, "-o", tmp, RATES_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building valu_rates")
    os.replace(tmp, RATES_BIN)
    return RATES_BIN


if __name__ == "__main__":
    print(build(verbose=True))

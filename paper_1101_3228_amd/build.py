"""Build the qtree HIP library (libqtree.so) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqtree.so")
BUILD = os.path.join(PKG, "_build")

SOURCES = ["api.cpp", "batch.cpp", "quantizer.cpp", "mlp_api.cpp", "fwd.hip", "count.hip",
           "bdp.hip", "diag.hip", "mlp.hip", "swing.hip", "lloyd.hip", "lloyd_api.cpp",
           "strat.hip", "fixed_scratch.hip", "buckets.hip"]

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


def _run(cmd, verbose: bool, what: str) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {what}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to an object in _build/ (in parallel), then link."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cflags = [f for f in FLAGS if f != "-shared"]
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1, 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_run, [hipcc(), *cflags, *inc, "-c", "-o", o,
                                 os.path.join(CSRC, s)], verbose, s)
                for s, o in zip(SOURCES, objs)]
        for f in futs:
            f.result()
    tmp = LIB + ".tmp"
    _run([hipcc(), *FLAGS, "-o", tmp, *objs], verbose, "libqtree.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

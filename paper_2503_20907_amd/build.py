"""Build libxrt.so (HIP for gfx950) in-tree.

    python -m paper_2503_20907_amd.build

Compiles every source under csrc/ with hipcc for gfx950 and links one shared
library next to this file.  Packed-FP32 instruction selection is disabled
(``-packed-fp32-ops``); FP32 arithmetic then issues as ordinary VALU ops.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libxrt.so")
SOURCES = ["xrt_kernels.hip", "xrt_api.cpp", "xrt_learn.hip", "xrt_learn.cpp", "xrt_batch.cpp",
           "xrt_noalloc.hip", "xrt_calib.hip"]
ARCH = os.environ.get("XRT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libxrt.so)")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-I", INCLUDE, "-I", CSRC]


def build(verbose: bool = False) -> str:
    """Compile and link; always rebuilds."""
    tmp = LIB + ".tmp%d" % os.getpid()
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc()] + flags() + ["-shared", "-o", tmp] + srcs + \
        ["-Wl,-rpath,/opt/rocm/lib", "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)

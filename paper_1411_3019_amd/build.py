"""Compile the HIP library libmd.so for gfx950 (in-tree)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "engine.hip")
LIB = os.path.join(PKG, "libmd.so")
HEADERS = [os.path.join(PKG, "csrc", "device.hpp"), os.path.join(PKG, "csrc", "kernels.hpp"),
           os.path.join(ROOT, "include", "md.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # FMA fusion only within one source expression, so that the step and the
    # finish kernels round identical expressions identically
    "-ffp-contract=on",
    # packed FP32 instructions stay disabled: only plain FP32/FP64 VALU forms are emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Always recompiles (the build check must exercise the compiler)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", tmp, SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libmd.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in [SRC, *HEADERS])


if __name__ == "__main__":
    print(build(verbose=True))

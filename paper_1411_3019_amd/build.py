"""Compile the HIP library libmd.so for gfx950 (in-tree).

The step kernels of each force class are separate translation units
(csrc/step_*.hip) compiled in parallel with the engine (csrc/engine.hip), then
linked into one shared library."""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmd.so")
OBJDIR = os.path.join(PKG, "_build")


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def headers() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hpp"))) + [os.path.join(ROOT, "include", "md.h")]


HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # FMA fusion only within one source expression, so that the step and the
    # finish kernels round identical expressions identically
    "-ffp-contract=on",
    # packed FP32 instructions stay disabled: only plain FP32/FP64 VALU forms are emitted
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src: str) -> tuple[str, subprocess.CompletedProcess]:
    obj = os.path.join(OBJDIR, os.path.splitext(os.path.basename(src))[0] + ".o")
    res = subprocess.run(["hipcc", *HIPCC_FLAGS, "-c", "-o", obj, src], capture_output=True, text=True)
    return obj, res


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Always recompiles (the build check must exercise the compiler)."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, srcs))
    objs = []
    for (obj, res), src in zip(results, srcs):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed compiling " + os.path.basename(src))
        if verbose:
            sys.stderr.write(res.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    res = subprocess.run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs],
                         capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libmd.so")
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in [*sources(), *headers()])


if __name__ == "__main__":
    print(build(verbose=True))

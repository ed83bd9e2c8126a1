"""Compile the gfx950 HIP library (csrc/) into libapcloud.so, in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libapcloud.so")
SOURCES = ["primitives.hip", "build.hip", "gfd.hip", "gfd4.hip", "sell.hip", "solve.hip",
           "learned.hip", "batch.hip", "push.hip", "noalloc.hip", "quad2d.hip", "api.cpp"]


def build_library(verbose: bool = False, jobs: int = 0) -> str:
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        # -packed-fp32-ops: no packed-FP32 instructions anywhere in the device code
        # (the host pass warns that it does not know the feature)
        cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-c",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", os.path.join(HERE, "..", "include"),
               "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    jobs = jobs or min(len(cmds), os.cpu_count() or 1, 8)
    with ThreadPoolExecutor(jobs) as ex:
        for r in list(ex.map(lambda c: subprocess.run(c, check=True), cmds)):
            pass
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))

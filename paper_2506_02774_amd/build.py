"""Build libvoyager.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvoyager.so")
SOURCES = ["api.hip", "scene.hip", "lod.hip", "render.hip", "serve.hip", "walk.hip", "peaks.hip"]
HEADERS = ["vy_common.hpp", "sort.hpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _newer(target, deps):
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile every source (all of them when `force`) and link the library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = [os.path.join(os.path.dirname(HERE), "include", h) for h in ("vy.h", "vy_serve.h")]
    hdrs = [os.path.join(CSRC, h) for h in HEADERS] + inc
    objs = []
    for src in SOURCES:
        sp = os.path.join(CSRC, src)
        op = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(op)
        if force or _newer(op, [sp] + hdrs):
            cmd = [HIPCC, *FLAGS, "-c", sp, "-o", op]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force="--incremental" not in sys.argv, verbose=True)

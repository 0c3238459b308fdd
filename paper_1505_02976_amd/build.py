"""Build of the HIP library liblbm.so for gfx950 (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_api.cpp", "lbm_kernels.hip", "lbm_adjoint.hip", "lbm_step2.hip", "lbm3d.hip", "lbm_scratch.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions in device code: the device pass honours this target
    # feature (the host pass prints that it does not know it and ignores it)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one source expression, so the same node code
    # rounds identically in every kernel it is inlined into (one-step, two-step, batched)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, `jobs` at a time; 0: one per source, at most 8)
    and link liblbm.so; returns its path."""
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds = []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmds.append([HIPCC] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    jobs = jobs or min(len(cmds), 8)
    running = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        running.append((cmd, subprocess.Popen(cmd)))
        while len(running) >= jobs:
            c, p = running.pop(0)
            if p.wait() != 0:
                raise subprocess.CalledProcessError(p.returncode, c)
    for c, p in running:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, c)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

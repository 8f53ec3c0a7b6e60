"""Compile the native parts in-tree: the input generators (gcc) and the HIP
library for gfx950 (hipcc).  Called by ``__graft_entry__.build()``; every call
recompiles."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")

HIP_SOURCES = [
    "ged_kernels.hip",
    "ged_api.hip",
    "ged_batch.hip",
    "ged_split.hip",
    "ged_spectral.hip",
    "ged_greedy.hip",
    "ged_server.hip",
    "ged_noalloc.hip",
]

HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    # packed fp32 instructions are disabled for every kernel in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-rdc",
]


def _run(cmd, cwd=None):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=cwd)


def build_inputs():
    src = os.path.join(PKG, "inputs", "graphgen.c")
    out = os.path.join(PKG, "inputs", "libgraphgen.so")
    _run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", src, "-o", out + ".tmp"])
    os.replace(out + ".tmp", out)
    return out


def build_hip(jobs: int = 8):
    out = os.path.join(PKG, "libged_hip.so")
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for s in HIP_SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(objdir, s.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [hipcc, *[f for f in HIP_FLAGS if f != "-shared"], "-c", "-I", INCLUDE, "-I", CSRC,
               src, "-o", obj]
        print("+", " ".join(cmd), flush=True)
        procs.append((s, subprocess.Popen(cmd)))
        if len(procs) >= jobs:
            s0, p0 = procs.pop(0)
            if p0.wait() != 0:
                raise RuntimeError(f"hipcc failed on {s0}")
    for s0, p0 in procs:
        if p0.wait() != 0:
            raise RuntimeError(f"hipcc failed on {s0}")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out + ".tmp",
          "-lpthread"])
    os.replace(out + ".tmp", out)
    return out


def build_all():
    build_inputs()
    build_hip()


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    {"inputs": build_inputs, "hip": build_hip, "all": build_all}[what]()

"""Host-side AddressSanitizer builds of the native parts, for the CPU tests
(never used by the GPU runs).  See build_asan()."""
from __future__ import annotations

import os
import sys

from ._build import CSRC, HIP_FLAGS, HIP_SOURCES, INCLUDE, PKG, ROOT, _run

LLVM = "/opt/rocm/llvm"
ASAN_RT = "libclang_rt.asan-x86_64.so"


def asan_runtime():
    """Path of clang's AddressSanitizer runtime, preloaded to run the CPU tests
    against the sanitized builds (Python itself is not instrumented)."""
    import glob
    hits = sorted(glob.glob(os.path.join(LLVM, "lib", "clang", "*", "lib", "linux", ASAN_RT)))
    if not hits:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return hits[-1]


def build_asan():
    """Host-side AddressSanitizer builds, in place of the normal ones: the input
    generators and the CPU oracle (clang, -fsanitize=address) and the HIP
    library with its host code sanitized (-Xarch_host, so no device code is
    instrumented).  Run the CPU tests under them with

        LD_PRELOAD=$(python -c 'from paper_1910_13874_amd import _build_asan as b; print(b.asan_runtime())') \
        ASAN_OPTIONS=detect_leaks=0 python -m pytest tests -m "not gpu"

    and rebuild the normal libraries (__graft_entry__.build()) afterwards."""
    clang = os.path.join(LLVM, "bin", "clang")
    san = ["-fsanitize=address", "-shared-libasan", "-fno-omit-frame-pointer", "-g", "-O1"]
    src = os.path.join(PKG, "inputs", "graphgen.c")
    out = os.path.join(PKG, "inputs", "libgraphgen.so")
    _run([clang, *san, "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", src, "-o",
          out + ".tmp", f"-Wl,-rpath,{LLVM}/lib"])
    os.replace(out + ".tmp", out)
    src = os.path.join(ROOT, "oracle", "ged_oracle.c")
    out = os.path.join(ROOT, "oracle", "libged_oracle.so")
    _run([clang, *san, "-std=c11", "-fPIC", "-shared", "-Wall", src, "-o", out + ".tmp", "-lm"])
    os.replace(out + ".tmp", out)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(PKG, "_build", "asan")
    os.makedirs(objdir, exist_ok=True)
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-shared-libasan",
                "-Xarch_host", "-fno-omit-frame-pointer", "-g"]
    objs = []
    for s in HIP_SOURCES:
        obj = os.path.join(objdir, s.replace(".hip", ".o"))
        _run([hipcc, *[f for f in HIP_FLAGS if f != "-shared"], *host_san, "-c", "-I", INCLUDE,
              "-I", CSRC, os.path.join(CSRC, s), "-o", obj])
        objs.append(obj)
    out = os.path.join(PKG, "libged_hip.so")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *host_san, *objs, "-o",
          out + ".tmp", "-lpthread"])
    os.replace(out + ".tmp", out)



if __name__ == "__main__":
    build_asan()

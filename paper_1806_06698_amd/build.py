"""Build libsyev3.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1806_06698_amd.build

compiles every source under csrc/ into paper_1806_06698_amd/libsyev3.so.
hipcc cross-compiles for gfx950 without a GPU present.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsyev3.so")

SOURCES = ["syev3_kernels.hip", "syev3_noalloc.hip", "syev3_api.cpp", "syev3_server.cpp"]

ARCH = os.environ.get("SYEV3_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # explicit fma() only: results do not depend on where the compiler
    # would have contracted, so every kernel computes bitwise the same
    "-ffp-contract=off",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libsyev3.so)")


def build(verbose: bool = False) -> str:
    """Compile every source and link libsyev3.so; always rebuilds."""
    cc = hipcc()
    with tempfile.TemporaryDirectory(prefix="syev3_build_") as tmp:
        objs = []
        for src in SOURCES:
            path = os.path.join(CSRC, src)
            obj = os.path.join(tmp, src + ".o")
            cmd = [cc, *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", path, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            p = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
            if p.returncode != 0:
                sys.stderr.write(p.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            if verbose:
                sys.stderr.write(p.stderr)
            objs.append(obj)
        out_tmp = LIB + ".tmp"
        rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(cc))), "lib")
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs,
               "-L" + rocm_lib, "-Wl,-rpath," + rocm_lib, "-lrocprofiler-sdk-roctx",
               "-lpthread"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

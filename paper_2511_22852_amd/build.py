"""Builds libccake_hip.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2511_22852_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libccake_hip.so")
DRIVER = os.path.join(PKG, "ccake_bench")
SOURCES = ["binning.hip", "stage.hip", "kernels.hip", "runtime.cpp", "server.cpp", "noalloc.hip"]
ARCH = os.environ.get("CCAKE_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
    # no packed FP32 instructions (v_pk_*_f32) anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        out = _run(["hipcc", *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
        if verbose and out:
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    # native driver of the C ABI (no Python in the process) with the same
    # objects linked into the executable: the counter profiler collects per
    # dispatch only for kernels of the executable's own code objects
    main_obj = os.path.join(BUILD, "ccake_bench.o")
    _run(["hipcc", *HIPCC_FLAGS, "-c", os.path.join(CSRC, "ccake_bench.cpp"), "-o", main_obj])
    tmp = DRIVER + ".tmp"
    _run(["hipcc", f"--offload-arch={ARCH}", "-o", tmp, main_obj, *objs, "-lpthread"])
    os.replace(tmp, DRIVER)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

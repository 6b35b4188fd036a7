"""Build step of libcmflb: compiles the HIP sources for gfx950 into
``libcmflb.so`` inside the package directory (in-tree, so the library
travels with the source tree)."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/cmflb_kernels.hip", "csrc/cmflb_capi.hip"]
ARCH = "gfx950"


def library_path():
    return os.path.join(HERE, "libcmflb.so")


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


def compile_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are disabled on purpose for every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # multiply-adds fused only within a source expression: every kernel
        # that inlines the collision (single lattice, ensemble) then rounds
        # identically, so replicas are bit-identical to standalone lattices
        "-ffp-contract=on",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"),
    ]


def link_flags():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return [f"-L{rocm}/lib", "-lhipfft", f"-Wl,-rpath,{rocm}/lib"]


def build(verbose=False):
    out = library_path()
    tmp = out + ".tmp"
    cmd = ([hipcc()] + compile_flags() + [os.path.join(HERE, s) for s in SOURCES] + link_flags()
           + ["-o", tmp])
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))

"""Build step of libcmflb: compiles the HIP sources for gfx950 into
``libcmflb.so`` inside the package directory (in-tree, so the library
travels with the source tree).

Each source is compiled in two passes: the device pass (gfx950 code object,
built with packed FP32 instructions disabled) and the host pass, which
embeds that code object; then the host objects are linked.  Splitting the
passes keeps device-only code-generation options away from the host
compiler.  Sources compile in parallel."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["csrc/cmflb_step_pull.hip", "csrc/cmflb_step_aa.hip", "csrc/cmflb_ensemble.hip",
           "csrc/cmflb_kernels.hip", "csrc/cmflb_capi.hip"]
ARCH = "gfx950"


def library_path():
    return os.path.join(HERE, "libcmflb.so")


def rocm_path():
    return os.environ.get("ROCM_PATH", "/opt/rocm")


def hipcc():
    for cand in (os.environ.get("HIPCC"), os.path.join(rocm_path(), "bin/hipcc"),
                 shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


def clangxx():
    cand = os.path.join(rocm_path(), "lib/llvm/bin/clang++")
    if os.path.exists(cand):
        return cand
    raise RuntimeError(f"{cand} not found: the two-pass build needs ROCm's clang++")


def compile_flags():
    """Flags shared by the device and the host pass."""
    return [
        "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # multiply-adds fused only within a source expression: every kernel
        # that inlines the collision (single lattice, ensemble) then rounds
        # identically, so replicas are bit-identical to standalone lattices
        "-ffp-contract=on",
        "-Wall", "-Wno-unused-function",
        "-I", os.path.join(ROOT, "include"),
    ]


def device_flags():
    # packed FP32 instructions are disabled on purpose for every kernel
    return ["--offload-device-only", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def link_flags():
    rocm = rocm_path()
    return [f"-L{rocm}/lib", "-lhipfft", f"-Wl,-rpath,{rocm}/lib"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=False):
    out = library_path()
    tmp = out + ".tmp"
    with tempfile.TemporaryDirectory(prefix="cmflb_build_") as work:
        srcs = [os.path.join(HERE, s) for s in SOURCES]
        stems = [os.path.join(work, os.path.splitext(os.path.basename(s))[0]) for s in srcs]
        dev = [[clangxx()] + compile_flags() + device_flags() + ["-c", s, "-o", st + ".gpu"]
               for s, st in zip(srcs, stems)]
        host = [[clangxx()] + compile_flags() +
                ["--offload-host-only", "-Xclang", "-fcuda-include-gpubinary",
                 "-Xclang", st + ".gpu", "-c", s, "-o", st + ".host.o"]
                for s, st in zip(srcs, stems)]
        with ThreadPoolExecutor(max_workers=len(srcs)) as pool:
            list(pool.map(lambda c: _run(c, verbose), dev))
            list(pool.map(lambda c: _run(c, verbose), host))
        _run([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] +
             [st + ".host.o" for st in stems] + link_flags() + ["-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))

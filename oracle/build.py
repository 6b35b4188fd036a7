"""Build step of the CPU oracle: compiles ``cmflb_oracle.c`` with gcc (FP64,
IEEE semantics: no fast-math) into ``liboracle.so`` beside it."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path():
    return os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    src = os.path.join(HERE, "cmflb_oracle.c")
    out = library_path()
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the FP64 CPU oracle (test infrastructure) into oracle/liborc.so with gcc.

Portable x86-64 code (no -march=native): the shared object may run on another host.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "velb_oracle.c")
    out = os.path.join(_HERE, "liborc.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

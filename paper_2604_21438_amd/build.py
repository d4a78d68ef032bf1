"""Build the gfx950 library libsfchem.so in-tree with hipcc.

Every HIP translation unit is compiled with packed FP32 instructions
disabled (-target-feature -packed-fp32-ops); the host pass reports that it
does not know the feature, which is expected.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libsfchem.so")
BUILD = os.path.join(ROOT, "_build")

SOURCES = ["sfk_li.hip", "sfk_serve.hip", "sfsched.cpp", "sfserve.cpp", "sfchem.cpp"]
# Extra device flags per source.  The LI kernels run one cell per lane for
# thousands of loop iterations; machine LICM hoists every loop-invariant
# binary64 constant (and products of them) out of that loop into registers,
# which doubles the kernel's VGPR use and halves its occupancy.
EXTRA = {"sfk_li.hip": ["-mllvm", "-disable-machine-licm"],
         "sfk_serve.hip": ["-mllvm", "-disable-machine-licm"]}
ARCH = os.environ.get("SFC_OFFLOAD_ARCH", "gfx950")

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + INCLUDE, "-I" + CSRC]


def build(verbose: bool = False) -> str:
    """Compile all sources and link libsfchem.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc", *FLAGS, *EXTRA.get(src, []), *lang, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the gfx950 library libsfchem.so in-tree with hipcc.

Every HIP translation unit is compiled with packed FP32 instructions
disabled (-target-feature -packed-fp32-ops); the host pass reports that it
does not know the feature, which is expected.

The build fails if a kernel spills vector registers to scratch memory: the
per-lane cell loops are written to keep every per-cell value in registers,
and a spill means a change has pushed a kernel over its register budget
(a decision to make explicitly, with a launch bound, not by accident).
Spills of scalar registers (into vector register lanes) are allowed.
"""
from __future__ import annotations

import os
import re
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


def vgpr_spills(remarks: str) -> dict:
    """Kernels with a non-zero 'VGPRs Spill' in hipcc's resource-usage
    remarks, with the count."""
    out, name = {}, None
    for ln in remarks.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", ln)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"remark:\s+VGPRs Spill: (\d+)", ln)
        if m and name and int(m.group(1)) > 0:
            out[name] = int(m.group(1))
    return out


def build(verbose: bool = False) -> str:
    """Compile all sources and link libsfchem.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmd = ["hipcc", *FLAGS, *EXTRA.get(src, []), *lang,
               "-Rpass-analysis=kernel-resource-usage", "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        other = [ln for ln in r.stdout.splitlines() if "kernel-resource-usage" not in ln]
        if other and (verbose or r.returncode != 0):
            print("\n".join(other), file=sys.stderr)
        if r.returncode != 0:
            raise subprocess.CalledProcessError(r.returncode, cmd)
        spilled = vgpr_spills(r.stdout)
        if spilled:
            raise RuntimeError(f"{src}: kernels spill vector registers: {spilled}")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


PROBE_SRC = os.path.join(ROOT, "tests", "math_probe.hip")
PROBE_LIB = os.path.join(ROOT, "tests", "libmathprobe.so")


def build_probe(verbose: bool = False) -> str:
    """The tests' probe of the kernels' binary64 math (tests/math_probe.hip)."""
    tmp = PROBE_LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-shared", "-o", tmp, PROBE_SRC]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        print(r.stdout, file=sys.stderr)
        raise subprocess.CalledProcessError(r.returncode, cmd)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


if __name__ == "__main__":
    print(build(verbose=True))

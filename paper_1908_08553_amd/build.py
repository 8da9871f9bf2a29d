"""Build step: compile the HIP/C++ sources into the in-tree shared library.

    python paper_1908_08553_amd/build.py

produces ``paper_1908_08553_amd/libtn.so`` for gfx950 with hipcc.  Packed
FP32 instructions are disabled for device code (``-packed-fp32-ops``).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtn.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-Wno-unused-result",
          "-I", INCLUDE, "-I", CSRC]
# Per-source device flags.  The register-resident chunk kernel keeps its
# whole slice in VGPRs: with MFMA results in the VGPR form the input and
# output tiles of a step share one register file (the AGPR form puts them in
# different files and doubles the footprint).
EXTRA = {"absorb_chunk_reg.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.cpp")) +
                  glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False) -> str:
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    cmds = []
    objs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        extra = EXTRA.get(os.path.basename(src), [])
        cmds.append([HIPCC, *COMMON, "-x", "hip", *DEVICE_FLAGS, *extra, "-c", src, "-o", obj])
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16))

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(jobs) as pool:
        list(pool.map(compile_one, cmds))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-pthread", *DEVICE_FLAGS, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

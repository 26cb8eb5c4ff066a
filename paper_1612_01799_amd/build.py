"""Compile the HIP/C++ sources of the solver into ``libpsn.so`` (gfx950).

Run ``python paper_1612_01799_amd/build.py`` (by path: importing the package
loads the library) or call :func:`build_library`.
Every call recompiles.  The library lands next to this file so that it
travels with the source tree.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpsn.so")
ARCH = "gfx950"

SOURCES = ["psn_passes_f32.hip", "psn_passes_f64.hip", "psn_passes_split.hip", "psn_general_f32.hip",
           "psn_general_f64.hip", "psn_kbuild.hip", "psn_plan.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # code-object v5: loadable by the HIP runtime bundled with PyTorch
    "-mcode-object-version=5",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _hipcc():
    for c in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build_library(verbose: bool = False, jobs: int = 7) -> str:
    hipcc = _hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {src}\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-mcode-object-version=5", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    # radix-16 microbenchmark (VALU butterflies vs MFMA), run by bench.py
    exe = os.path.join(HERE, "dft16_valu_vs_mfma")
    cmd = [hipcc, *FLAGS, "-x", "hip", os.path.join(CSRC, "microbench", "dft16_valu_vs_mfma.hip"), "-o", exe + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: dft16_valu_vs_mfma\n{r.stdout}\n{r.stderr}")
    os.replace(exe + ".tmp", exe)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))

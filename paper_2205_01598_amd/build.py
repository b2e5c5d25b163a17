"""Build ``libmpk.so`` in-tree for gfx950.

Host planner: g++ with OpenMP.  Kernels and C-ABI: hipcc for gfx950 only,
with packed-FP32 instructions disabled.  The shared library links the HIP
runtime directly; PyTorch is not involved.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmpk.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPCC_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-result"]
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-Wall", "-Wno-unused-function"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    jobs = [
        ["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, "plan.cpp"), "-o", os.path.join(BUILD, "plan.o")],
        [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "mpk_device.hip"),
         "-o", os.path.join(BUILD, "mpk_device.o")],
        [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "mlp.hip"), "-o", os.path.join(BUILD, "mlp.o")],
        [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, "plan_device.hip"),
         "-o", os.path.join(BUILD, "plan_device.o")],
    ]
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        list(ex.map(lambda c: _run(c, verbose), jobs))
    tmp = LIB + ".tmp"
    _run(["g++", "-shared", "-fopenmp", "-o", tmp, os.path.join(BUILD, "plan.o"),
          os.path.join(BUILD, "mpk_device.o"), os.path.join(BUILD, "mlp.o"), os.path.join(BUILD, "plan_device.o"),
          f"-L{ROCM}/lib", "-lamdhip64",
          f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Builds libocck.so in-tree for gfx950 (hipcc for the HIP kernels, amdclang++
for the host C++).  ``python -m paper_1708_05353_amd.build`` or build()."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libocck.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in ordinary VGPRs: without it the GEMM K loops copy
    # their accumulators between AGPRs and VGPRs on every iteration
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-ffp-contract=off", "-Wall", "-Wno-unused-function"]

HIP_SOURCES = ["far_k.hip", "batch.hip", "selector.hip", "far_j.hip", "near_k.hip"]
CXX_SOURCES = ["tree_build.cpp", "abi.cpp"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd)}")
    return r


def build(verbose: bool = False) -> str:
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    cxx = os.path.join(ROCM, "llvm", "bin", "clang++")
    jobs = []
    for src in HIP_SOURCES:
        jobs.append([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", os.path.join(bdir, src + ".o")])
    for src in CXX_SOURCES:
        jobs.append([cxx, *CXX_FLAGS, f"-I{ROCM}/include", "-c", os.path.join(CSRC, src),
                     "-o", os.path.join(bdir, src + ".o")])
    objs = [j[-1] for j in jobs]
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda cmd: _run(cmd, verbose), jobs))
    tmp = OUT + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

"""Build libhelm.so (HIP kernels for gfx950 + host C++) in the package folder.

    python -m paper_2004_06309_amd.build

Host sources are compiled with amdclang++ (OpenMP, AVX2), HIP sources with
hipcc for gfx950; objects go to ``_build/`` at the repository root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libhelm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["fem.cpp", "decomp.cpp", "order.cpp", "factor_gpu.cpp", "coarse.cpp", "solver.cpp", "api.cpp"]
HIP_SOURCES = ["device.hip", "device_block.hip", "device_factor.hip", "device_bgmres.hip"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result", f"-I{ROCM}/include", f"-I{ROOT}/include"]
HOST_FLAGS = COMMON + ["-D__HIP_PLATFORM_AMD__", "-fopenmp", "-mavx2", "-mfma", "-ffp-contract=fast"]
HIP_FLAGS = COMMON + ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                      "-munsafe-fp-atomics"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{p.stdout}")
    return p.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    jobs = []
    objs = []
    for s in HOST_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([clang, *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        objs.append(o)
        jobs.append([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fopenmp", "--offload-arch=gfx950", "-o", tmp, *objs,
          f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", f"-Wl,-rpath,{ROCM}/llvm/lib"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

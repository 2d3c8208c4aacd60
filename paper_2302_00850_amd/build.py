"""Build libcola.so (HIP kernels for gfx950 + the C-ABI host library) in-tree.

    python -m paper_2302_00850_amd.build

Objects go to paper_2302_00850_amd/_build/, the library to
paper_2302_00850_amd/libcola.so.  Packed FP32 instructions are disabled for
all device code (-packed-fp32-ops): the compiler otherwise forms them from
plain float arithmetic.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcola.so")
ARCH = os.environ.get("COLA_OFFLOAD_ARCH", "gfx950")

SOURCES = ["hop_f64_18.hip", "hop_f64_12.hip", "hop_f32_12.hip", "hop_f16_12.hip", "hop_flic.hip", "hop_dispatch.cpp", "pack.hip", "blas.hip", "blas_block.hip", "clover.hip", "force.hip", "hmc.hip", "hmc_driver.cpp", "ops.cpp", "solver.cpp",
           "scratch.hip", "eigen_vec.hip", "eigen.cpp", "api.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-Wno-unused-command-line-argument", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", f"--offload-arch={ARCH}", "-I", os.path.join(HERE, "..", "include")]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip() and verbose:
        print(r.stderr, file=sys.stderr)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))

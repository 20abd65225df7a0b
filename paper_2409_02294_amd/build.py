"""Compile the HIP sources under ``csrc/`` into ``libps.so`` for gfx950.

Each translation unit is compiled by ``hipcc`` in parallel into ``_build/``
and linked into ``paper_2409_02294_amd/libps.so`` (in-tree, so a copy of the
tree carries the built library).  Usage: ``python -m paper_2409_02294_amd.build``.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libps.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-mcode-object-version=5",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    # .cpp sources hold host code only (the ABI layer): no device pass
    host_only = ["--offload-host-only"] if src.endswith(".cpp") else []
    cmd = [HIPCC, "-x", "hip", *COMMON, *host_only, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    build_example()
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources, and {EXAMPLE}")
    return LIB


EXAMPLE = os.path.join(HERE, "examples", "solve_c")
ROCM = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))


def build_example() -> str:
    """The plain-C caller of the ABI (examples/solve_c.c), linked against the
    in-tree libps.so and the HIP runtime (no torch)."""
    src = EXAMPLE + ".c"
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", src, "-o", EXAMPLE,
           "-I", os.path.join(os.path.dirname(HERE), "include"), "-I", os.path.join(ROCM, "include"),
           "-D__HIP_PLATFORM_AMD__", "-L", HERE, "-lps", "-Wl,-rpath,$ORIGIN/..",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"example build failed:\n{r.stderr}")
    return EXAMPLE


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build the package's native libraries in-tree.

* libhive.so          -- the HIP kernels and the C ABI declared in include/hive.h
                          (hipcc, gfx950 only);
* libworkload_gen.so  -- the seeded workload generator (gcc, OpenMP).

Run as `python -m paper_2510_15095_amd.build`.  Every call recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
ARCH = "gfx950"

HIP_SOURCES = ["hive.hip", "hash_study.hip", "gather.hip"]
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # packed fp32 forms are disabled for all HIP code built here
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd: list[str]) -> None:
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def _atomic_replace(tmp: str, dst: str) -> None:
    os.replace(tmp, dst)


def build_workload() -> str:
    out = os.path.join(PKG, "libworkload_gen.so")
    tmp = out + ".tmp"
    _run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall",
          os.path.join(CSRC, "workload_gen.c"), "-lm", "-o", tmp])
    _atomic_replace(tmp, out)
    return out


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def build_hive() -> str:
    out = os.path.join(PKG, "libhive.so")
    tmp = out + ".tmp"
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES]
    _run([hipcc(), *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp])
    _atomic_replace(tmp, out)
    return out


def build_all() -> None:
    build_workload()
    build_hive()


if __name__ == "__main__":
    what = sys.argv[1:] or ["all"]
    for w in what:
        {"all": build_all, "workload": build_workload, "hive": build_hive}[w]()

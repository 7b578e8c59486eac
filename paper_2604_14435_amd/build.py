"""Build the gfx950 HIP library ``libdvq.so`` in-tree with hipcc.

    python -m paper_2604_14435_amd.build          # compile + link
    python -m paper_2604_14435_amd.build --check  # print the command lines only

Every source is compiled for gfx950 only.  Packed FP32 instructions are
disabled for all device code (``-target-feature -packed-fp32-ops``).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdvq.so")

SOURCES = [
    "api_common.hip",
    "decompose.hip",
    "circuits.hip",
    "circuits_fast.hip",
    "cost.hip",
    "adjoint.hip",
    "adjoint_fast.hip",
    "mlp.hip",
    "mlp_fused.hip",
]

DEVICE_FLAGS = [
    "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
COMMON_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-I", INCLUDE]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libdvq.so)")


def compile_cmd(src: str) -> list[str]:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    return [hipcc(), *COMMON_FLAGS, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]


def link_cmd() -> list[str]:
    objs = [os.path.join(BUILD, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    return [hipcc(), "-shared", "-fPIC", *DEVICE_FLAGS, *objs, "-o", LIB + ".tmp"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source and link ``libdvq.so``; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    cmds = [compile_cmd(s) for s in SOURCES]
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 2)))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed ({r.returncode}):\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return r.stderr

    with cf.ThreadPoolExecutor(jobs) as ex:
        for err in ex.map(run, cmds):
            if verbose and err.strip():
                print(err, file=sys.stderr)
    run(link_cmd())
    os.replace(LIB + ".tmp", LIB)
    return LIB


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--check", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    if a.check:
        for s in SOURCES:
            print(" ".join(compile_cmd(s)))
        print(" ".join(link_cmd()))
        return
    print(build(verbose=a.verbose))


if __name__ == "__main__":
    main()

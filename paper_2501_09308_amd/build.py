"""Builds libxrdvi.so (HIP, gfx950) in the package directory.

    python -m paper_2501_09308_amd.build [--save-temps DIR]
"""
from __future__ import annotations

import argparse
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libxrdvi.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-fvisibility=hidden",
    # packed FP32 instructions are not generated (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I", INCLUDE, "-I", CSRC,
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip"))
                  + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(save_temps: str | None = None, verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    for src in sources():
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if save_temps:
            os.makedirs(save_temps, exist_ok=True)
            cmd.insert(1, f"-save-temps={'obj'}")
            cmd[cmd.index("-o") + 1] = os.path.join(save_temps, os.path.basename(obj))
            obj = cmd[cmd.index("-o") + 1]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs,
           "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


UBENCH_SRC = os.path.join(PKG, "ubench", "ubench.hip")
UBENCH_LIB = os.path.join(PKG, "ubench", "libxrdvi_ubench.so")


def build_ubench(verbose: bool = False) -> str:
    """Instruction-rate microbenchmarks (a separate library)."""
    cmd = [HIPCC, *FLAGS, "-shared", UBENCH_SRC, "-o", UBENCH_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(UBENCH_LIB + ".tmp", UBENCH_LIB)
    return UBENCH_LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--save-temps", default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args(argv)
    print(build(a.save_temps, a.verbose))
    print(build_ubench(a.verbose))


if __name__ == "__main__":
    sys.exit(main())

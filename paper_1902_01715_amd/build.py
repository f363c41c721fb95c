"""Build step of the HIP library: compiles csrc/ for gfx950 into libaspamg.so (in-tree).

Solve kernels are built with contraction allowed (FMA); the setup kernels and
the host decision code with -ffp-contract=off so that their sums are the
sequential IEEE sums they are written as.  Packed-FP32 instruction selection is
disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libaspamg.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = os.environ.get("ASPAMG_ARCH", "gfx950")
COMMON = ["-O3", "-fPIC", "-std=c++17", f"-I{INCLUDE}", f"-I{CSRC}", "-Wall",
          "-Wno-unused-result", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]

SOURCES = [
    # (file, is_device, extra flags)
    ("kernels_solve.hip", True, []),
    ("kernels_setup.hip", True, ["-ffp-contract=off"]),
    ("kernels_coarsen.hip", True, ["-ffp-contract=off"]),
    ("kernels_batch.hip", True, []),
    ("noalloc.hip", True, []),
    ("batch_api.cpp", False, []),
    ("setup_host.cpp", False, ["-ffp-contract=off", "-fopenmp"]),
    ("api.cpp", False, ["-fopenmp"]),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"compile failed: {cmd[-1]}")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src, dev, extra in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = ["hipcc", "-c", path, "-o", obj] + COMMON + extra
        cmd += DEVICE if dev else [f"--offload-arch={ARCH}"]
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-fopenmp", "-lamdhip64"]
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

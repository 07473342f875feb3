"""Build libfactory_sdf.so for gfx950 with hipcc, in-tree.

    python -m paper_2205_03532_amd.build

Always recompiles.  Objects go to ``paper_2205_03532_amd/_build/``; the shared
library to ``paper_2205_03532_amd/libfactory_sdf.so``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libfactory_sdf.so")
BUILD = os.path.join(PKG, "_build")
ARCH = os.environ.get("FC_OFFLOAD_ARCH", "gfx950")

# -ffp-contract=off: every FMA in the kernels is an explicit fmaf, so all code
# paths evaluating a query round identically.  Packed FP32 instructions are
# disabled for the device code.
DEVICE_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]
HOST_FLAGS = ["--cuda-host-only", f"--offload-arch={ARCH}", "-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]


def _hipcc():
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found")
    return h


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"build step failed ({r.returncode}): {' '.join(cmd[:3])} ...")
    if verbose and (r.stdout or r.stderr):
        print((r.stdout + r.stderr)[-4000:], flush=True)


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src in ("fc_kernels.hip", "fc_patches.hip", "fc_bake.hip"):
        objs.append(os.path.join(BUILD, src.replace(".hip", ".o")))
        _run([hipcc, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", objs[-1]], verbose)
    objs.append(os.path.join(BUILD, "fc_api.o"))
    _run([hipcc, *HOST_FLAGS, "-c", os.path.join(CSRC, "fc_api.cpp"), "-o", objs[-1]], verbose)
    tmp = OUT + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
          "-Wl,-rpath,/opt/rocm/lib"], verbose)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

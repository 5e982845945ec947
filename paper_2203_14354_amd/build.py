"""Build the gfx950 transport library ``libxephot.so`` in-tree with hipcc.

Device code is compiled for gfx950 only, with packed-FP32 instruction
selection disabled (``-packed-fp32-ops``), multiply-add fusion limited to
single expressions (``-ffp-contract=on``, so that all kernel instantiations
round alike), FP32 division and square root from the hardware approximations
(``-fno-hip-fp32-correctly-rounded-divide-sqrt``; a few ulp, far inside the
parity tolerances) and hardware floating-point atomics
(``-munsafe-fp-atomics``) for the FP64 gradient tallies.
"""
from __future__ import annotations

import os
import shutil
import concurrent.futures
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libxephot.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HOST_SOURCES = ["api.cpp", "bvh.cpp"]
DEVICE_SOURCES = ["propagate.hip", "propagate_tally.hip"]
ARCH = "gfx950"


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("command failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    os.makedirs(BUILD_DIR, exist_ok=True)
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]
    # -ffp-contract=on: multiply-adds fuse only within one expression, so every
    # instantiation of the transport kernel rounds identically
    # -fno-hip-fp32-correctly-rounded-divide-sqrt: FP32 division and square root
    # by the hardware reciprocal/root instructions (a few ulp) instead of the
    # multi-instruction correctly rounded sequences
    # -fgpu-flush-denormals-to-zero: FP32 denormals flush to zero, so the library
    # math left on the path (logarithms, rare-branch divisions) needs no range
    # scaling for them; no value on the transport path is that small
    dev = ["-x", "hip", f"--offload-arch={ARCH}", "-munsafe-fp-atomics", "-ffp-contract=on",
           "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
    srcs = HOST_SOURCES + DEVICE_SOURCES
    objs = [os.path.join(BUILD_DIR, s + ".o") for s in srcs]
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(srcs)) as pool:
        list(pool.map(lambda so: _run([hipcc, *common, *dev, "-c", os.path.join(CSRC, so[0]),
                                       "-o", so[1]]), zip(srcs, objs)))
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

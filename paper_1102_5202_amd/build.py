"""Build ``libgrmhd.so`` (HIP, gfx950) in-tree.

    python -m paper_1102_5202_amd.build

All device code is compiled with packed-FP32 instruction selection disabled
(``-packed-fp32-ops``) and without fast-math (no reassociation, infinities
and NaNs honoured); FMA contraction is left at the compiler default.
Single-precision division and square root (used only by the mixed-precision
path's face physics and sources) take the hardware reciprocal and
square-root instructions instead of the correctly rounded sequences
(``-fno-hip-fp32-correctly-rounded-divide-sqrt``: a few ulp of FP32, far
below that path's FP32 rounding of the states).  Double-precision division
is a reciprocal refined by two Newton steps times the numerator instead of
the correctly rounded division sequence (``-freciprocal-math
-fapprox-func`` on the device side: within 2 ulp, about 4 fewer
instructions per division; 1.5 % on a step, measured); double square roots
are unchanged.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libgrmhd.so")
SOURCES = ["grmhd_kernels.hip", "grmhd_adjoint.hip", "grmhd_api.hip", "grmhd_batch.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-hip-fp32-correctly-rounded-divide-sqrt",
         "-Xarch_device", "-freciprocal-math", "-Xarch_device", "-fapprox-func",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, extra=()) -> str:
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp,
           *[os.path.join(CSRC, s) for s in SOURCES]]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libgrmhd.so")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

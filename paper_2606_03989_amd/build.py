"""Builds libpixvod.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled with packed FP32 instructions disabled; the
library links the ROCm HIP runtime. Python users load it through
paper_2606_03989_amd, which imports torch first so that both share one HIP
runtime.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpixvod.so")
SOURCES = ["gbp_kernels.hip", "gbp_adjoint.hip", "gbp_tree.hip", "gbp_transfer.hip", "pixvod_runtime.hip", "pixvod_unroll.hip", "pixvod_central.hip"]
ARCH = os.environ.get("PIXVOD_ARCH", "gfx950")

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-source flags. The persistent passes in gbp_kernels.hip loop over tiles
# around a body that needs every register: hoisting loop-invariant values
# (constants, addresses) out of such a loop only makes them spill, so machine
# loop-invariant code motion is off there.
SOURCE_FLAGS = {"gbp_kernels.hip": ["-mllvm", "-disable-machine-licm"]}
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result"]


def build(verbose: bool = False, jobs: int = 4) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [hipcc, *COMMON, *DEVICE_FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), cmd))
        objs.append(obj)
    for p, cmd in procs:
        if p.wait() != 0:
            raise RuntimeError("compilation failed: " + " ".join(cmd))
    tmp = LIB + ".tmp"
    link = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
            "-Wl,-rpath,/opt/rocm/lib", "-Wl,-soname,libpixvod.so"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

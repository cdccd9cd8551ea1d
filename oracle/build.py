"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

gcc -O2 with OpenMP and without fast-math, so that the oracle keeps IEEE
double semantics.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Builds the oracle into `out`. `defines` (NAME=VALUE strings) is for the
    tests' planted-fault variants only; the oracle itself is built without."""
    src = os.path.join(HERE, "pixvod_oracle.c")
    tmp = out + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
           "-D_DEFAULT_SOURCE", *[f"-D{d}" for d in defines], "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

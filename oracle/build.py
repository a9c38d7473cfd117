"""Compile the oracle's C source into two shared libraries (FP64 and long double).

The oracle is test infrastructure: only the test suite, the smoke check and the CPU-baseline leg
of the benchmark load what this builds.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
TARGETS = {
    "liboracle.so": [],
    "liboracle_ld.so": ["-DOG_LONG_DOUBLE"],
}
# IEEE arithmetic: no -ffast-math, no contraction of a*b+c into fused multiply-adds.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]


def build(verbose: bool = False) -> None:
    for name, extra in TARGETS.items():
        out = os.path.join(HERE, name)
        cmd = ["gcc", *CFLAGS, *extra, SRC, "-o", out + ".tmp", "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

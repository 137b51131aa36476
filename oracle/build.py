"""Build the CPU oracle shared libraries (test infrastructure only).

Two builds of the same plain-C source:
  liboracle_f64.so  -- REAL = double (the oracle)
  liboracle_q.so    -- REAL = __float128 (the oracle's own accuracy check)
Portable x86-64 code (no -march=native: the library may run on another
host), IEEE arithmetic (no -ffast-math), OpenMP over shellsets.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mdx_oracle.c")


def build(verbose: bool = False) -> None:
    common = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-Wall",
              "-Wno-unused-function", "-Wno-unused-variable"]
    jobs = [
        (common + [SRC, "-o", os.path.join(HERE, "liboracle_f64.so"), "-lm"]),
        (common + ["-DORACLE_QUAD", SRC, "-o", os.path.join(HERE, "liboracle_q.so"),
                   "-lquadmath", "-lm"]),
    ]
    for cmd in jobs:
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)

"""Builds the CPU oracle shared library (test infrastructure only).

Plain gcc, binary64 with contraction off so that every product and sum is
rounded as written; binary128 through libquadmath for the per-observation
remainder; OpenMP over particles only.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "subsmc_oracle.c")
LIB = os.path.join(HERE, "liboracle_subsmc.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
        "-o", LIB + ".tmp", SRC, "-lquadmath", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Compile the CPU oracle into oracle/libebboracle.so with gcc.

Test infrastructure: the oracle is built by the project's build step so that
the tests and the benchmark's CPU-baseline leg can load it; the GPU library
never links or calls it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libebboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "ebb_oracle.c")
    # -ffp-contract=off: no fused multiply-add, so every product and sum is
    # rounded as written (the Morton quantisation relies on it).
    # -fopenmp: only the *_mt timing entries use threads.
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

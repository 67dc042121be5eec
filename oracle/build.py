"""Build the oracle shared library (plain C, gcc, FP64, no fused multiply-add,
OpenMP over independent groups).

Test infrastructure only: the oracle is built so that the test suite, the
smoke check and the benchmark's CPU-baseline leg can call it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pphd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-fopenmp", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

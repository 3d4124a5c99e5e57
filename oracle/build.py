"""Build the CPU oracle shared library (test infrastructure only).

g++ -O2 -ffp-contract=off (no FMA contraction, no fast-math) so the oracle's
arithmetic is exactly the expression trees written in ars_oracle.cpp.
OpenMP on the outer cell loops does not change any result: cell updates are
independent and the only reduction feeding the state (the time step) is a max.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ars_oracle.cpp")
LIB = os.path.join(HERE, "libars_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
        "-Wall", "-Wno-unused-function",
        SRC, "-o", LIB + ".tmp",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

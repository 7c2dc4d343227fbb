"""Compile the CPU oracle (test infrastructure) into oracle/liboracle_wandqs.so.

-O3 with OpenMP; no floating-point contraction, so every operation rounds as
written.  The code is built for the generic x86-64 target, so the same library
runs on any host it is copied to; -ffp-contract=off and the absence of
-ffast-math keep the results independent of the target's vector width.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wandqs_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_wandqs.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

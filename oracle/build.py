"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

gcc -O2 -ffp-contract=off keeps every floating-point operation of the index
rule and of the accumulations rounded exactly as written (no fused
multiply-add contraction).  OpenMP is enabled for the band-parallel
gridder used for the CPU rate (orc_grid_window_par); every other function is
single-threaded."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC",
           "-fopenmp", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

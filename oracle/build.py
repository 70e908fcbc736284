"""Compile the CPU oracle (plain C, OpenMP) into oracle/_lmep_oracle.so.

Test infrastructure: the oracle is built so the tests, the smoke check and the
CPU-baseline leg of the benchmark can load it; nothing in the product calls it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lmep_oracle.c")
OUT = os.path.join(HERE, "_lmep_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unused-function",
           SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=HERE)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

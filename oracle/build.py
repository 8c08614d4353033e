"""Build the CPU oracle shared library (test infrastructure only).

Compiles ``oracle_dd.c`` with gcc into ``liboracle_dd.so`` next to it.
``-ffp-contract=off`` keeps the compiler from fusing the multiply-adds that
the error-free transformations depend on; FMA is used only where the source
calls ``fma()`` explicitly (TwoProduct).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle_dd.c")
LIB = os.path.join(HERE, "liboracle_dd.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-mfma", "-mavx2",
        "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

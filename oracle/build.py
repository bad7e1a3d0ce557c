"""Build step for the FP64 CPU oracle (test infrastructure).

Compiles ``pond_oracle.c`` with gcc into ``liboracle_pond.so`` next to it:
plain C99, OpenMP over destination nodes, no fast-math and no floating-point
contraction, so every product and sum rounds as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pond_oracle.c")
LIB = os.path.join(HERE, "liboracle_pond.so")

CFLAGS = ["-std=c99", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    """Compile the oracle library and return its path (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Compile the C oracle into ``oracle/libsgml_oracle.so`` with gcc.

TEST INFRASTRUCTURE: builds the checker, never part of the product path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sgml_oracle.c")
LIB = os.path.join(HERE, "libsgml_oracle.so")


def build(verbose: bool = False) -> str:
    # -O2 without -ffast-math: the oracle keeps IEEE FP64 semantics.
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

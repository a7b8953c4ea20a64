"""Compile the C oracle into oracle/liblbm_oracle.so (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose: bool = False) -> str:
    # -ffp-contract=off: no fused multiply-add, so every product is rounded
    # exactly as written (vectorisation without fast-math
    # does not reorder sums, so the results do not depend on -O or -march).
    # x86-64-v3 (AVX2) rather than -march=native: the library is built on one
    # machine and run on another, whose CPU may lack this one's extensions.
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-Wall", "-Wextra", SRC, "-o", LIB, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

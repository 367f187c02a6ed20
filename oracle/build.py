"""Compile the oracle's C library (test infrastructure only)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", SO,
           os.path.join(HERE, "bmm_oracle.c")]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose=True)

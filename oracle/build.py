"""Build the oracle's plain-C kernels (``lbm_ref.c``) into ``liblbm_ref.so``.

TEST INFRASTRUCTURE ONLY: the oracle is the correctness reference for the HIP
solver and is never part of the product path."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_ref.c")
OUT = os.path.join(HERE, "liblbm_ref.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", SRC, "-o", OUT + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

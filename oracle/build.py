"""Builds the C oracle (``ref.c``) into ``liboracle.so`` next to this file.

Plain gcc, FP64, OpenMP.  ``-ffp-contract=off`` keeps the compiler from fusing
multiplies and adds on its own: the only fused multiply-adds in the oracle are
the explicit ``fma()`` calls in the K-means distance.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(HERE, "ref.c")
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-shared", "-fPIC", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

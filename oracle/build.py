"""Compile the FP64 oracle into ``oracle/liboo_oracle.so`` with gcc.

Strict IEEE double arithmetic: no fast-math and no FMA contraction, so the
oracle's rounding is that of the plain C expressions. OpenMP only spreads
independent queries over threads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    src = os.path.join(HERE, "octaoctree_oracle.c")
    out = os.path.join(HERE, "liboo_oracle.so")
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", out + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

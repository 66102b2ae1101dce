"""Compile the FP64 CPU oracle into oracle/libcplb_ref.so (test infrastructure).

Plain gcc, OpenMP over node loops, no floating-point contraction so that
every multiply and add rounds exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcplb_ref.so")


def build(verbose=False):
    src = os.path.join(HERE, "cplb_ref.c")
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Compile the FP64 CPU oracle into oracle/libcplb_ref.so (test infrastructure).

Plain gcc, OpenMP over node loops, no floating-point contraction so that
every multiply and add rounds exactly as written (and no reassociation:
-O3 vectorises only where the order of every sum is kept, so the results
are those of -O0).  The target is x86-64-v3 (AVX2) rather than the build
host's own instruction set: the library is built once and also run on
other hosts, whose CPUs may lack the build host's AVX-512 extensions.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libcplb_ref.so")


def build(verbose=False):
    src = os.path.join(HERE, "cplb_ref.c")
    cmd = ["gcc", "-std=c11", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

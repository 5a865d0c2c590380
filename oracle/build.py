"""Builds the CPU oracle (test infrastructure only) into oracle/liboracle.so.

Plain gcc, -O2, no fast-math, no FMA contraction, OpenMP over packets.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "smcrt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    lib_t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > lib_t
               for f in ("smcrt_oracle.c", "smcrt_oracle.h"))


if __name__ == "__main__":
    print(build(verbose=True))

"""Build step for the CPU oracle (test infrastructure).

Compiles oracle/sdcsz_ref.cpp into oracle/libsdcsz_ref.so with g++, strict
IEEE arithmetic: no fused multiply-add contraction, no fast math, SSE2
scalar math (the x86-64 default), so every float operation is one rounded
IEEE operation in the order the source writes it.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sdcsz_ref.cpp")
LIB = os.path.join(HERE, "libsdcsz_ref.so")

FLAGS = ["-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
         "-Wall", "-Wextra"]


def build(verbose=False):
    cmd = ["g++"] + FLAGS + ["-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the FP64 CPU oracle (test infrastructure only) into oracle/liborc.so.

Plain g++ build: no contraction, no fast-math, OpenMP only over independent blocks.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["orc_euler.cpp", "orc_mr.cpp", "orc_riemann.cpp", "orc_tree.cpp", "orc_mlp.cpp",
           "orc_schemes.cpp", "orc_tait.cpp", "orc_viscous.cpp"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the CPU oracle library (test infrastructure) with g++.

The oracle is plain C++ compiled for a generic x86-64-v3 host so the same
shared object runs on any AVX2 machine.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libwh_oracle.so")
SOURCES = [os.path.join(HERE, "wh_oracle.cpp"), os.path.join(HERE, "gbs.cpp")]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["g++", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC", "-std=c++17",
           "-Wall", "-Wno-unused-function", "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

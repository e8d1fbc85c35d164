"""Build the CPU oracle library (test infrastructure) with g++.

The oracle is plain C++ compiled for a generic x86-64-v3 host so the same
shared object runs on any AVX2 machine.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libwh_oracle.so")
SOURCES = [os.path.join(HERE, "wh_oracle.cpp"), os.path.join(HERE, "gbs.cpp")]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    """sanitize: an AddressSanitizer + UndefinedBehaviorSanitizer build (for
    the sanitizer tier of the tests; load it with the sanitizer runtimes
    preloaded and WH_ORACLE_LIB pointing at it)."""
    lib = out or LIB
    tmp = lib + ".tmp"
    if sanitize:
        opt = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    else:
        opt = ["-O3", "-march=x86-64-v3"]
    cmd = ["g++"] + opt + ["-fopenmp", "-shared", "-fPIC", "-std=c++17",
                           "-Wall", "-Wno-unused-function", "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

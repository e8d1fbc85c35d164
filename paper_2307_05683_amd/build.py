"""Compile the HIP library libwh.so for gfx950 (in-tree, with hipcc)."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "wh.hip")
LIB = os.path.join(PKG, "libwh.so")
ARCH = os.environ.get("WH_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=" + ARCH,
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", os.path.join(PKG, "csrc"),
]


PROBE_SRC = os.path.join(PKG, "csrc", "fp64_issue_probe.hip")
PROBE = os.path.join(PKG, "fp64_issue_probe")


def _hipcc(cmd, out, verbose):
    tmp = out + ".tmp"
    cmd = cmd + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, out)


def build(verbose: bool = False, extra=()) -> str:
    _hipcc(["hipcc"] + FLAGS + list(extra) + [SRC], LIB, verbose)
    # the FP64 issue-rate probe bench.py reports beside the roofline (a
    # standalone program, not part of the library)
    probe_flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    _hipcc(["hipcc"] + probe_flags + [PROBE_SRC], PROBE, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

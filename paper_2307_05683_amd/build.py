"""Compile the HIP library libwh.so for gfx950 (in-tree, with hipcc)."""
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "wh.hip")
PAIR_SRC = os.path.join(PKG, "csrc", "wh_pair_step.hip")
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
# The pair layout's step kernel (wh_pair_step.hip) is scheduled for
# instruction latency rather than occupancy: at 242 VGPRs, two resident
# wavefronts per SIMD (three with the default schedule), it measured 1.6-2.4%
# faster on 65536 eight-planet systems with GR, while the one-planet and split
# kernels in wh.hip, one wavefront per SIMD in their launches, measured
# slower with it.
PAIR_FLAGS = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]


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
    # two translation units compiled side by side, then linked into one
    # shared library (each object carries its own gfx950 code object)
    cflags = [f for f in FLAGS if f != "-shared"] + list(extra)
    with tempfile.TemporaryDirectory() as tmp:
        jobs = []
        for src, more in ((SRC, []), (PAIR_SRC, PAIR_FLAGS)):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            # a fixed compilation-unit id: the default one hashes the
            # temporary object path, which would make every build differ
            cuid = "-cuid=" + os.path.splitext(os.path.basename(src))[0]
            cmd = ["hipcc", "-c", cuid] + cflags + more + [src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        failed = False
        for obj, proc in jobs:
            out, _ = proc.communicate()
            if proc.returncode != 0:
                sys.stderr.write(out)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed")
        _hipcc(["hipcc", "-shared", "-fPIC", "--offload-arch=" + ARCH] + [o for o, _ in jobs], LIB, verbose)
    # the FP64 issue-rate probe bench.py reports beside the roofline (a
    # standalone program, not part of the library)
    probe_flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    _hipcc(["hipcc"] + probe_flags + [PROBE_SRC], PROBE, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

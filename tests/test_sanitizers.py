"""Sanitizer builds of the CPU code (AddressSanitizer + UndefinedBehavior-
Sanitizer, every finding fatal).

* The library's host logic (wh_host.h: lane packings, workspace layout,
  configuration checks, SABA_n coefficients, tape sizes, launch windows) is
  compiled with g++ alone into a checking program, run here.
* The oracle is rebuilt with the sanitizers and its pin tests run against it
  in a child process with the sanitizer runtimes preloaded.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM_INC = "/opt/rocm/include"


def _runtime(name):
    p = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


need_gxx = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@need_gxx
def test_host_logic_under_sanitizers(tmp_path):
    if not os.path.exists(os.path.join(ROCM_INC, "hip", "hip_runtime_api.h")):
        pytest.skip("HIP headers not available")
    exe = str(tmp_path / "host_logic_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2307_05683_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "host_logic_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0"))
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0 and "host logic ok" in r.stdout


@need_gxx
def test_oracle_pins_under_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not available")
    sys.path.insert(0, ROOT)
    from oracle import build as oracle_build
    lib = oracle_build.build(sanitize=True, out=str(tmp_path / "libwh_oracle_asan.so"))
    env = dict(os.environ, WH_ORACLE_LIB=lib, LD_PRELOAD=asan + " " + ubsan,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_kepler.py", "test_oracle_substeps.py",
                                                       "test_oracle_map.py", "test_oracle_jacobi.py",
                                                       "test_oracle_saba.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu"] + tests,
                       capture_output=True, text=True, timeout=1200, env=env, cwd=ROOT)
    print(r.stdout[-3000:], r.stderr[-3000:])
    assert r.returncode == 0
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr

"""The library's host code (planning, argument checks, the tuning-table
parser, the host M-Basis and matrix inverse, the batched layout) and the
oracle, built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven through every path that runs before device work
(tests/sanitize/driver.cpp). CPU only: the device code is linked unchanged
and never launched."""
from __future__ import annotations

import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_04356_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_1905_04356_amd", "_build")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer", "-g", "-O1"]


def test_host_code_and_oracle_under_asan_and_ubsan(tmp_path):
    if not os.path.exists(CLANG):
        pytest.skip("clang++ with the sanitizer runtimes is not installed")
    hip_objs = sorted(glob.glob(os.path.join(BUILD, "*.hip.o")))
    if not hip_objs:
        pytest.skip("device objects not built (run the package build first)")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
           "-D__HIP_PLATFORM_AMD__"]
    jobs, objs = [], []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        objs.append(obj)
        jobs.append([CLANG, "-x", "c++", "-std=c++17", "-fPIC"] + SAN + inc + ["-c", src, "-o", obj])
    orc = str(tmp_path / "pm_oracle.o")
    objs.append(orc)
    jobs.append([CLANG, "-x", "c", "-std=c11"] + SAN +
                ["-c", os.path.join(ROOT, "oracle", "pm_oracle.c"), "-o", orc])
    drv = str(tmp_path / "driver.o")
    objs.append(drv)
    jobs.append([CLANG, "-std=c++17"] + SAN + inc +
                ["-c", os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), "-o", drv])
    procs = [(j, subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
             for j in jobs]
    for j, pr in procs:
        out, _ = pr.communicate(timeout=600)
        assert pr.returncode == 0, " ".join(j) + "\n" + out
    exe = str(tmp_path / "driver")
    link = [CLANG] + SAN + objs + hip_objs + ["-o", exe, "-L/opt/rocm/lib", "-lamdhip64",
                                              "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", PM_TUNE_TABLE="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "sanitized host driver: ok" in r.stdout

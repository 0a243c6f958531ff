"""Build libpm.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_1905_04356_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libpm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed fp32 instructions are turned off for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) +
                  glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
               "-Wall", "-I", INCLUDE, "-c", src, "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = DEVICE_FLAGS
        else:
            # host-only translation unit: plain C++ against the HIP runtime
            cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I",
                   "/opt/rocm/include"] + cmd[2:]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                            stderr=subprocess.STDOUT, text=True)))
        if len(procs) >= jobs:
            _wait(procs, verbose)
            procs = []
    _wait(procs, verbose)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed: " + " ".join(cmd))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def _wait(procs, verbose):
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        noise = [ln for ln in out.splitlines()
                 if "packed-fp32-ops' is not a recognized feature" not in ln]
        if verbose and noise:
            sys.stdout.write("\n".join(noise) + "\n")
        if p.returncode != 0:
            sys.stderr.write("\n".join(noise) + "\n")
            failed.append(" ".join(cmd))
    if failed:
        raise RuntimeError("compile failed:\n" + "\n".join(failed))


if __name__ == "__main__":
    build(verbose=True)

"""Build the CPU oracle shared library with gcc (test infrastructure only).

    python oracle/build.py            # -> oracle/liborc.so
    python oracle/build.py --plant 3  # -> a mutant with planted mistake 3

The oracle is compiled from pm_oracle.c alone; it links nothing from the GPU
library.
"""
from __future__ import annotations

import argparse
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pm_oracle.c")


def build(out: str | None = None, plant: int = 0, quiet: bool = True) -> str:
    out = out or os.path.join(HERE, "liborc.so")
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
           f"-DORC_PLANT={int(plant)}", SRC, "-o", out + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("oracle build failed: " + " ".join(cmd))
    os.replace(out + ".tmp", out)
    if not quiet:
        print("built", out)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--plant", type=int, default=0)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    build(a.out, a.plant, quiet=False)

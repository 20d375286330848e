"""Build the HIP shared library libgalkin.so for gfx950, in-tree.

    python paper_2205_06819_amd/build.py

(run by path: importing the package would load the library being rebuilt).

Compiles paper_2205_06819_amd/csrc/galkin.hip with hipcc into
paper_2205_06819_amd/libgalkin.so.  Packed FP32 instructions are disabled
(``-packed-fp32-ops``); the host pass warns that it does not know that
target feature, which is harmless.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgalkin.so")
ARCH = os.environ.get("GALKIN_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC)")


def build(verbose: bool = False) -> str:
    src = os.path.join(CSRC, "galkin.hip")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", "-shared", "-fPIC", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{res.stderr[-8000:]}")
    errs = [l for l in res.stderr.splitlines() if ": error:" in l]
    if errs:
        raise RuntimeError("\n".join(errs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    path = build(verbose=True)
    print(path)

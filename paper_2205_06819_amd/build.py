"""Build the HIP shared library libgalkin.so for gfx950, in-tree.

    python paper_2205_06819_amd/build.py

(run by path: importing the package would load the library being rebuilt).

Compiles the translation units under paper_2205_06819_amd/csrc with hipcc in
parallel and links them into paper_2205_06819_amd/libgalkin.so:

* galkin.hip      host side of the C ABI, HMC update and data-preparation kernels;
* fwd_inst.hip    the single-grid forward kernel, once per (mode, PSF mode) pair;
* multi_inst.hip  the many-grid forward kernel, once per PSF mode;
* adj.hip         the adjoint kernel, once per PSF mode.

Packed FP32 instructions are disabled (``-packed-fp32-ops``); the host pass
warns that it does not know that target feature, which is harmless.

``build_sanitized_harness()`` also links tests/sanitize/abi_check.cpp against
the host translation unit compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: each -fsanitize flag goes after
-Xarch_host) and the kernel objects of the normal build, into
paper_2205_06819_amd/_build/abi_check_asan (run by tests/test_sanitize.py).
The objects are kept in paper_2205_06819_amd/_build/.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgalkin.so")
OBJDIR = os.path.join(HERE, "_build")
HARNESS = os.path.join(OBJDIR, "abi_check_asan")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
ARCH = os.environ.get("GALKIN_ARCH", "gfx950")

# (object name, source, extra defines)
UNITS = [("galkin", "galkin.hip", [])]
UNITS += [(f"fwd_m{m}_l{l}", "fwd_inst.hip", [f"-DGK_MODE={m}", f"-DGK_LW={l}"]) for m in (0, 1, 2) for l in (0, 1)]
UNITS += [(f"multi_l{l}", "multi_inst.hip", [f"-DGK_LW={l}"]) for l in (0, 1)]
UNITS += [(f"adj_l{l}_k{k}", "adj.hip", [f"-DGK_LW={l}", f"-DGK_KH={k}"]) for l in (0, 1) for k in (4, 6)]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC)")


def _flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = [l for l in res.stderr.splitlines() if ": error:" in l]
    if res.returncode != 0 or errs:
        raise RuntimeError(f"{' '.join(cmd[:2])} ... failed ({res.returncode}):\n{res.stderr[-8000:]}")
    return res


def build(verbose: bool = False, jobs: int = 0) -> str:
    cc = hipcc()
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    os.makedirs(OBJDIR, exist_ok=True)
    cmds = []
    for name, src, defs in UNITS:
        obj = os.path.join(OBJDIR, name + ".o")
        cmds.append([cc, *_flags(), *defs, "-c", os.path.join(CSRC, src), "-o", obj])
    if verbose:
        for c in cmds:
            print(" ".join(c), file=sys.stderr)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    out = LIB + ".tmp"
    link = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}",
            *[os.path.join(OBJDIR, n + ".o") for n, _, _ in UNITS], "-o", out]
    if verbose:
        print(" ".join(link), file=sys.stderr)
    _run(link)
    os.replace(out, LIB)
    return LIB


def build_sanitized_harness(verbose: bool = False) -> str:
    """The ABI check program with the host code under ASan/UBSan (needs the
    kernel objects of build())."""
    cc = hipcc()
    kern = [os.path.join(OBJDIR, n + ".o") for n, _, _ in UNITS if n != "galkin"]
    if not all(os.path.exists(k) for k in kern):
        build(verbose)
    host = os.path.join(OBJDIR, "galkin_asan.o")
    check = os.path.join(OBJDIR, "abi_check_asan.o")
    cmds = [[cc, *_flags(), "-O1", "-g", *SAN, "-c", os.path.join(CSRC, "galkin.hip"), "-o", host],
            [cc, *_flags(), "-O1", "-g", *SAN, "-c", os.path.join(ROOT, "tests", "sanitize", "abi_check.cpp"),
             "-o", check]]
    with ThreadPoolExecutor(max_workers=2) as ex:
        list(ex.map(_run, cmds))
    out = HARNESS + ".tmp"
    _run([cc, f"--offload-arch={ARCH}", *SAN, check, host, *kern, "-o", out])
    os.replace(out, HARNESS)
    return HARNESS


if __name__ == "__main__":
    path = build(verbose="-v" in sys.argv)
    print(path)
    if "--harness" in sys.argv:
        print(build_sanitized_harness(verbose="-v" in sys.argv))

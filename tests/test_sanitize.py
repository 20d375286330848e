"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(tests/sanitize/abi_check.cpp, linked by build.build_sanitized_harness with
the sanitizers on host code only): argument validation on the CPU; on a GPU
also grid creation, the set_data host path, shape rules, the batched calls,
the many-grid plan cache and the allocation-free entry point's limit."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "paper_2205_06819_amd", "_build", "abi_check_asan")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _harness():
    if not os.path.exists(HARNESS):
        import importlib.util
        spec = importlib.util.spec_from_file_location("galkin_build", os.path.join(ROOT, "paper_2205_06819_amd",
                                                                                   "build.py"))
        mod = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(mod)
        mod.build_sanitized_harness()
    return HARNESS


def _run(env):
    r = subprocess.run([_harness()], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-3000:], flush=True)
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    assert r.returncode == 0, out[-3000:]
    return out


def test_abi_validation_under_sanitizers():
    # no device visible: the harness checks argument validation only
    out = _run(dict(ENV, HIP_VISIBLE_DEVICES="-1"))
    assert "validation only" in out


@pytest.mark.gpu
def test_abi_device_paths_under_sanitizers():
    print("case: sanitized host ABI harness with the GPU", flush=True)
    out = _run(ENV)
    assert "device checks" in out

"""The C ABI's host code (argument checks, planner, workspace layout, the
allocation-free entry point's validation, status strings) under AddressSanitizer
and UndefinedBehaviorSanitizer: the library is built with both on its host
code (device code unchanged), the ASan runtime is preloaded into a fresh
interpreter, and the CPU ABI tests run against that build.  Any sanitizer
report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_1611_05677_amd import build as build_mod  # noqa: E402


@pytest.mark.slow
def test_abi_tests_pass_under_host_sanitizers():
    if build_mod.is_stale(build_mod.LIB_HOSTSAN):
        build_mod.build_host_sanitized()
    rt = build_mod.asan_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env.update({"LD_PRELOAD": rt, "FMG_LIBRARY": build_mod.LIB_HOSTSAN,
                # the interpreter itself is not instrumented: its allocations are
                # not leaks of the library; any other report aborts the run
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    res = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-q",
                          "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert " passed" in out

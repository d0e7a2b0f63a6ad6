"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: the CPU tests of the C ABI (argument checks,
status strings, batch requirements, null handling) run in a child process
against the sanitizer build (paper_2106_15214_amd/build.py, build_sanitized),
with the shared sanitizer runtime preloaded.  Any sanitizer report fails."""
import os
import subprocess
import sys

import pytest

from paper_2106_15214_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_tests_clean_under_asan_and_ubsan():
    rt = build.sanitizer_runtime()
    if not rt:
        pytest.skip("no shared AddressSanitizer runtime in /opt/rocm/llvm")
    try:
        lib = build.build_sanitized()
    except RuntimeError as e:  # pragma: no cover - toolchain without hipcc
        pytest.skip(str(e))
    env = dict(os.environ)
    env.update({
        "NMF_BETA_LIBRARY": lib,
        "LD_PRELOAD": rt,
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi_cpu.py"), "-q",
                        "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "runtime error" not in out and "Sanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out

"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Two child processes run CPU test files against sanitizer builds of the same
sources: the C ABI's host side (argument checks, plans, work lists and the
limit checks of the allocation-free entry point, built with clang's
sanitizers for the host only) under tests/test_abi.py, and the oracle (built
with gcc's) under its pins.  Any report fails the child and so this test.
No GPU is used: every call in those files fails validation before a HIP call
or runs on the host.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OPTS = "detect_leaks=0:abort_on_error=1:halt_on_error=1:verify_asan_link_order=0"


def _run(files, env_extra):
    env = dict(os.environ, ASAN_OPTIONS=OPTS, UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               **env_extra)
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                          "-p", "no:cacheprovider"] + files,
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]
    return out


def test_c_abi_host_code_under_asan_ubsan():
    from paper_1503_06202_amd import build

    lib = build.build_sanitized()
    rt = build.asan_runtime()
    if not rt:
        pytest.skip("clang AddressSanitizer runtime not found")
    out = _run(["tests/test_abi.py"], {"XENG_LIBRARY": lib, "LD_PRELOAD": rt})
    assert " passed" in out


def test_oracle_under_asan_ubsan():
    import oracle.build as ob

    lib = ob.build(sanitize=True)
    rt = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.isabs(rt):
        pytest.skip("gcc AddressSanitizer runtime not found")
    out = _run(["tests/test_oracle_pins.py"], {"ORACLE_LIBRARY": lib, "LD_PRELOAD": rt,
                                               "OMP_NUM_THREADS": "4"})
    assert " passed" in out

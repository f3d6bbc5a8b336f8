"""The CPU ABI tests (argument validation, error paths, plan creation without a
device) against a host AddressSanitizer + UndefinedBehaviorSanitizer build of the
library (tests/sanitized_build.py).  Any sanitizer report ends the run and fails
the test.  CPU only: the instrumented build is never loaded on a GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_tests_pass_under_host_sanitizers():
    pytest.importorskip("torch")
    from tests import sanitized_build as sb
    lib = sb.build()  # about a minute when the sources changed
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms, "the library is not instrumented"
    env = dict(os.environ, LD_PRELOAD=sb.runtime(), SLRX_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0:detect_odr_violation=0:"
                            "verify_asan_link_order=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    assert " passed" in r.stdout, out

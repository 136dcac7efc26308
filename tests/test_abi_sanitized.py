"""CPU: the C-ABI's host-side validation under AddressSanitizer and
UndefinedBehaviorSanitizer.  Every library source is built with both on its
host code (device code as usual) and linked with tests/abi_host_check.cpp,
which calls the entry points with invalid arguments (null pointers, sides and
indices out of range, bad options, staging beyond the no-allocation array)
and checks the returned status and message; any sanitizer report (memory
error, leak, undefined behaviour) fails the run.  No GPU is touched."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_validation_is_clean_under_sanitizers():
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("host-validation program: runs only without a GPU")
    from paper_2607_00579_amd import build
    exe = build.build_host_check()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "abi host checks passed" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr

"""The host-side ABI checks (test_abi_host.py) re-run against a build of the
ABI layer instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only; the kernels are the normal objects), in a child process
that preloads the sanitizer runtime.  CPU only: no compute call runs."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_host_checks_under_address_and_ub_sanitizers():
    from paper_1712_00238_amd import build as B
    try:
        lib = B.build_host_sanitized()
        rt = B.sanitizer_runtime()
    except RuntimeError as e:  # no hipcc / no kernel objects in this checkout
        pytest.skip(str(e))
    env = dict(os.environ, SDF_LIB_PATH=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out

"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the host-sanitized library (paper_1509_06820_amd/build_sanitized.py:
the host side of every source instrumented, device code as usual) and runs
the CPU checks of the C ABI (tests/test_capi_cpu.py: symbol exports,
workspace queries including random and extreme sizes, argument rejection)
against it in a subprocess with the ASan runtime preloaded.  Any sanitizer
report ends the subprocess with an error.  Needs no GPU: every call made
there returns before launching anything.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _toolchain():
    from paper_1509_06820_amd import build, build_sanitized
    return all(os.path.exists(p) or shutil.which(p) for p in (build.HIPCC, build_sanitized.CLANG))


@pytest.mark.skipif(not _toolchain(), reason="hipcc / clang++ not available")
def test_c_abi_host_code_is_sanitizer_clean():
    from paper_1509_06820_amd import build_sanitized as bs
    if bs.stale():
        bs.build_sanitized()
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": bs.asan_runtime(),
        "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
        "RQRCP_LIB": bs.LIB,
    })
    # -s: a sanitizer report goes to fd 2, which pytest would otherwise capture
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_capi_cpu.py"), "-q", "-x", "-s",
           "-p", "no:cacheprovider", "-m", "not gpu"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out

"""The host-side C++ of the library (argument checks, solver drivers,
workspace layout, the index self-test) under AddressSanitizer and
UndefinedBehaviorSanitizer: a build of the host sources with both
sanitizers (device code uninstrumented) runs the ABI tests in a child
process with the sanitizer runtimes preloaded.  Any report fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if p.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_abi_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    from paper_2303_08609_amd import build
    lib = build.build_sanitized()
    env = dict(os.environ, WILSON_EO_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=99",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=98")
    code = ("import sys, pytest; from paper_2303_08609_amd import wilson_eo as W; W.load(); "
            "assert 'libwilson_eo_san' in open('/proc/self/maps').read(); "
            "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', 'tests/test_abi.py']))")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]

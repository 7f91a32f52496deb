"""AddressSanitizer and UndefinedBehaviorSanitizer on the CPU: the oracle
through a driver that calls every one of its entry points on small lattices,
and the library's host code (argument validation, sizes, status strings, NULL
contexts, context creation) through the C ABI. No GPU is used: where no GPU
is present, context creation must fail cleanly."""
import os
import subprocess

import pytest

from sanitize import build as sb

pytestmark = pytest.mark.slow

ENV = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers(tmp_path):
    assert "oracle driver: ok" in _run(sb.build_oracle(str(tmp_path)))


def test_library_host_code_under_sanitizers(tmp_path):
    assert "abi driver: ok" in _run(sb.build_abi(str(tmp_path)))

"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/sanitize_driver.cpp calls every entry point of the C ABI; it is
linked with the library's sources compiled with the sanitizers on their host
code only (tests/native/build_sanitized.py), so that argument validation, the
workspace layouts, the operator schedules, tile timing, graph capture and the
no-allocation path run instrumented.  Without a device the driver covers the
validation paths; with one it also runs small problems through every entry
point.  A sanitizer report, a leak or a failed check fails the test.
"""
import os
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "native"))
import build_sanitized as bs  # noqa: E402

# leaks whose allocation stack runs through the ROCm runtime are the runtime's own
SUPP = os.path.join(os.path.dirname(bs.DRIVER), os.pardir, "lsan.supp")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1",
           LSAN_OPTIONS=f"suppressions={os.path.abspath(SUPP)}:print_suppressions=0")


def _run(mode: str, timeout: int) -> str:
    print(f"sanitize_driver {mode}", flush=True)
    r = subprocess.run([bs.DRIVER, mode], capture_output=True, text=True, timeout=timeout, env=ENV)
    out = r.stdout + r.stderr
    for marker in ("AddressSanitizer", "LeakSanitizer", "runtime error"):
        assert marker not in out, out[-6000:]
    assert r.returncode == 0 and f"{mode} mode: 0 failure(s)" in out, out[-6000:]
    return out


def test_host_code_under_sanitizers_without_device():
    if bs.stale():
        bs.build()
    _run("cpu", 120)


@pytest.mark.gpu
def test_host_code_under_sanitizers_on_device():
    assert os.path.exists(bs.DRIVER), (
        f"{bs.DRIVER} is missing: build it with `python tests/native/build_sanitized.py`")
    out = _run("gpu", 600)
    assert "straggler phase" in out and "time reversal" in out

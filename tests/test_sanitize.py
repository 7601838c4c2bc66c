"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`python -m paper_2110_01716_amd.build_lib --sanitize` builds a copy of the
library with host-only instrumentation and the driver
tests/sanitize/sem_sanitize_driver.cpp. The CPU test checks that the driver is
instrumented (a planted heap overflow in its own host code is reported); the
GPU test runs the driver over the C ABI: mesh setup (gather-scatter map), pMG
setup (coarse entity keys), Schwarz setup (face maps), solves, batches,
projection, GMRES and the error paths. Both skip when the sanitized build is
absent or older than the sources it was built from.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "paper_2110_01716_amd", "_build_san")
DRIVER = os.path.join(SAN, "sem_sanitize_driver")
LIB_SOURCES = [os.path.join(ROOT, "paper_2110_01716_amd", "csrc", f)
               for f in os.listdir(os.path.join(ROOT, "paper_2110_01716_amd", "csrc"))] + \
              [os.path.join(ROOT, "include", "sem.h")]
DRIVER_SOURCE = os.path.join(ROOT, "tests", "sanitize", "sem_sanitize_driver.cpp")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0", UBSAN_OPTIONS="print_stacktrace=1")


def _built():
    if not os.path.exists(DRIVER):
        return "sanitized build absent (python -m paper_2110_01716_amd.build_lib --sanitize)"
    lib = os.path.join(SAN, "libsem_san.so")
    if not os.path.exists(lib):
        return "sanitized library absent"
    stale = [f for f in LIB_SOURCES if os.path.getmtime(f) > os.path.getmtime(lib)]
    if os.path.getmtime(DRIVER_SOURCE) > os.path.getmtime(DRIVER):
        stale.append(DRIVER_SOURCE)
    if stale:
        return f"sanitized build older than {os.path.basename(stale[0])}"
    return None


def test_sanitized_driver_is_instrumented():
    why = _built()
    if why:
        pytest.skip(why)
    r = subprocess.run([DRIVER, "--self-check"], capture_output=True, text=True, env=ENV, timeout=60)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr


@pytest.mark.gpu
def test_sanitized_driver_runs_clean():
    why = _built()
    if why:
        pytest.skip(why)
    print("CASE sanitized driver", flush=True)
    r = subprocess.run([DRIVER], capture_output=True, text=True, env=ENV, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ok (0 failures)" in out
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out

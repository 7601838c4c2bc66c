"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`python -m paper_2110_01716_amd.build_lib --sanitize` builds a copy of the
library with host-only instrumentation and the driver
tests/sanitize/sem_sanitize_driver.cpp. The CPU test checks that the driver is
instrumented (a planted heap overflow in its own host code is reported); the
GPU test runs the driver over the C ABI: mesh setup (gather-scatter map), pMG
setup (coarse entity keys), Schwarz setup (face maps), solves, batches,
projection, GMRES and the error paths. Both skip when the sanitized build is
absent or was built from sources whose contents have changed since (the build
records a digest of them).
"""
import os
import subprocess

import pytest

from paper_2110_01716_amd import build_lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = build_lib.BUILD_SAN
DRIVER = os.path.join(SAN, "sem_sanitize_driver")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0", UBSAN_OPTIONS="print_stacktrace=1")


def _built():
    if not os.path.exists(DRIVER) or not os.path.exists(os.path.join(SAN, "libsem_san.so")):
        return "sanitized build absent (python -m paper_2110_01716_amd.build_lib --sanitize)"
    if not os.path.exists(build_lib.SAN_DIGEST):
        return "sanitized build has no source digest (build it again)"
    with open(build_lib.SAN_DIGEST) as fh:
        if fh.read().strip() != build_lib.san_sources_digest():
            return "sanitized build is older than its sources (their contents changed since)"
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

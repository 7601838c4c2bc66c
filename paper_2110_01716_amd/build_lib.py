"""Build libsem.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2110_01716_amd.build_lib [--jobs N] [--debug] [--sanitize]

Every source under csrc/ is compiled with hipcc --offload-arch=gfx950 and
linked into paper_2110_01716_amd/libsem.so. Always rebuilds (the build check
must compile every time it is asked to).

--sanitize builds a second copy of the library with its host code under
AddressSanitizer and UndefinedBehaviorSanitizer (device code is not
instrumented) into _build_san/libsem_san.so, and the driver
tests/sanitize/sem_sanitize_driver.cpp linked against it into
_build_san/sem_sanitize_driver (run it on a machine with the GPU).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsem.so")
BUILD_SAN = os.path.join(PKG, "_build_san")
DRIVER_SAN = os.path.join(ROOT, "tests", "sanitize", "sem_sanitize_driver.cpp")
# host-only instrumentation: each sanitizer flag applies to the host pass alone
SAN_FLAGS = ["-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

ARCH = os.environ.get("SEM_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    # never emit packed FP32 arithmetic (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp")):
            out.append(os.path.join(CSRC, f))
    return out


def compile_one(src: str, extra: list[str], out_dir: str = BUILD) -> tuple[str, float]:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [hipcc(), *COMMON, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    t = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        warn = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if warn:
            sys.stderr.write("\n".join(warn[:40]) + "\n")
    return obj, time.time() - t


def build(jobs: int | None = None, debug: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    extra = ["-g"] if debug else []
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(compile_one, s, extra): s for s in srcs}
        for fu in cf.as_completed(futs):
            obj, dt = fu.result()
            objs.append(obj)
            if verbose:
                print(f"  compiled {os.path.basename(futs[fu])} in {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *sorted(objs), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"  linked {LIB}", flush=True)
    return LIB


SAN_DIGEST = os.path.join(BUILD_SAN, "sources.sha256")


def san_sources_digest() -> str:
    """SHA-256 over what the sanitized build is made from (library sources,
    the public header, the driver, this build script with its flags), by
    content: a checkout that only touches modification times leaves it
    unchanged."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    files = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))]
    files += [os.path.join(ROOT, "include", "sem.h"), DRIVER_SAN, os.path.abspath(__file__)]
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def build_sanitized(jobs: int | None = None, verbose: bool = True) -> str:
    """Host-ASan/UBSan copy of the library plus the driver that exercises it;
    records the digest of the sources it was built from."""
    os.makedirs(BUILD_SAN, exist_ok=True)
    if os.path.exists(SAN_DIGEST):
        os.remove(SAN_DIGEST)
    digest = san_sources_digest()
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(compile_one, s, SAN_FLAGS, BUILD_SAN): s for s in srcs}
        for fu in cf.as_completed(futs):
            obj, dt = fu.result()
            objs.append(obj)
            if verbose:
                print(f"  compiled {os.path.basename(futs[fu])} (sanitized) in {dt:.1f}s", flush=True)
    lib = os.path.join(BUILD_SAN, "libsem_san.so")
    drv_obj = os.path.join(BUILD_SAN, "sem_sanitize_driver.o")
    steps = [
        [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *SAN_FLAGS, *sorted(objs), "-o", lib],
        [hipcc(), *COMMON, *SAN_FLAGS, "-c", DRIVER_SAN, "-o", drv_obj],
        [hipcc(), f"--offload-arch={ARCH}", *SAN_FLAGS, drv_obj, lib, f"-Wl,-rpath,{BUILD_SAN}",
         "-o", os.path.join(BUILD_SAN, "sem_sanitize_driver")],
    ]
    for cmd in steps:
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"sanitized build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if san_sources_digest() != digest:
        raise RuntimeError("sanitized build: the sources changed while they were compiled; build again")
    with open(SAN_DIGEST, "w") as fh:
        fh.write(digest + "\n")
    if verbose:
        print(f"  linked {lib} and {os.path.join(BUILD_SAN, 'sem_sanitize_driver')}", flush=True)
    return lib


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--sanitize", action="store_true", help="host-sanitized library and driver (_build_san/)")
    a = ap.parse_args()
    if a.sanitize:
        build_sanitized(a.jobs)
    else:
        build(a.jobs, a.debug)


if __name__ == "__main__":
    main()

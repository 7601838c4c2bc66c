"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/sem.h declares, and its host-side reference operators (GLL points,
Dhat, Jhat) agree with the oracle. No GPU call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import reference_ops as ro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sem.h")
LIB = os.path.join(ROOT, "paper_2110_01716_amd", "libsem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sem_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is missing: run `python -m paper_2110_01716_amd.build_lib`")
    from paper_2110_01716_amd import sem
    return sem.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sem_mesh_create", "sem_ax", "sem_gs", "sem_pmg_setup", "sem_pcg_solve"):
        assert n in names
    assert len(names) >= 25


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(raw, n)]
    assert not missing, missing
    from paper_2110_01716_amd import sem
    assert set(declared_functions()) <= set(sem.exported_symbols())


@pytest.mark.parametrize("N", list(range(1, 16)))
def test_host_reference_operators_match_oracle(lib, N):
    from paper_2110_01716_amd import sem
    x, w, D = sem.sem_reference(N)
    xo, wo = ro.gll(N)
    np.testing.assert_allclose(x, xo, atol=2e-15)
    np.testing.assert_allclose(w, wo, rtol=1e-13)
    np.testing.assert_allclose(D, ro.deriv_matrix(N), atol=1e-12 * N * N)


@pytest.mark.parametrize("Nc,Nf", [(1, 7), (3, 7), (1, 3), (2, 5), (4, 9), (6, 8)])
def test_host_interpolation_matches_oracle(lib, Nc, Nf):
    from paper_2110_01716_amd import sem
    np.testing.assert_allclose(sem.sem_interpolation(Nc, Nf), ro.prolongation_1d(Nc, Nf), atol=1e-13)


def test_host_argument_errors(lib):
    from paper_2110_01716_amd import sem
    assert lib.sem_reference(0, None, None, None) == sem.SEM_EINVAL
    assert lib.sem_reference(16, None, None, None) == sem.SEM_EINVAL
    assert b"outside" in lib.sem_last_error()
    assert lib.sem_mesh_create(None, None) == sem.SEM_EINVAL
    assert lib.sem_status_string(sem.SEM_ENOCONV).startswith(b"SEM_ENOCONV")
    # bandwidth probe: argument checks happen before any device work
    assert lib.sem_stream(0, None, None, 1.0, 2, None) == sem.SEM_EINVAL
    assert lib.sem_stream(9, None, None, 1.0, 2, None) == sem.SEM_EINVAL
    assert lib.sem_stream(2, None, None, 1.0, 3, None) == sem.SEM_EINVAL
    assert lib.sem_stream(2, None, None, 1.0, 0, None) == sem.SEM_OK
    assert lib.sem_dot_noalloc(None, 0, None, None, None, None) == sem.SEM_EINVAL
    # mesh sizes: rejected before any array is read or any device call is made,
    # including element counts whose point count would overflow 64 bits
    import ctypes as C
    h = C.c_void_p()
    dummy = C.c_double(0.0)
    for N, E in ((0, 1), (16, 1), (7, 0), (7, 2 ** 22), (1, 2 ** 61)):
        d = sem.sem_mesh_desc(N=N, E=E, x=C.addressof(dummy), y=C.addressof(dummy), z=C.addressof(dummy),
                              gid=C.addressof(dummy))
        assert lib.sem_mesh_create(C.byref(d), C.byref(h)) == sem.SEM_EINVAL
        assert h.value is None
    assert b"2^31-1" in lib.sem_last_error()

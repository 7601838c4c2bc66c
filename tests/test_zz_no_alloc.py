"""The allocation-free inner product (sem_dot_noalloc) against sem_dot:
two calls in a row on one device, the second on a smaller mesh (the static
scratch keeps the first call's contents), in FP64 and FP32, then the first
mesh again."""
import numpy as np
import pytest

from paper_2110_01716_amd import workloads as wl

from gpu_util import dev, print_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2110_01716_amd import sem as s
    s.load()
    return s


def _case(sem, bm, seed, dtype):
    import torch
    m = sem.Mesh.from_box(bm)
    u = dev(wl.random_rhs(bm, seed)).to(dtype)
    v = dev(wl.random_rhs(bm, seed + 1)).to(dtype)
    ref = sem.sem_dot(m.h, u, v)
    scale = sem.sem_dot(m.h, u.abs(), v.abs())
    return m, u, v, ref, scale


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dot_noalloc_matches_dot(sem, dtype):
    import torch
    tdt = torch.float64 if dtype == "f64" else torch.float32
    print_case("dot-noalloc", dtype)
    big = wl.box_mesh(12, N=7, deform=0.05, seed=1002)       # 884,736 local points: two points per thread
    small = wl.box_mesh(3, 2, 2, N=5, deform=0.05, seed=7)   # 2,592 local points
    cases = [_case(sem, big, 31, tdt), _case(sem, small, 41, tdt)]
    cases.append(cases[0])
    for m, u, v, ref, scale in cases:
        got = sem.sem_dot_noalloc(m.h, u, v)
        assert abs(got - ref) <= 1e-13 * scale, (got, ref)
        assert got == sem.sem_dot_noalloc(m.h, u, v)  # deterministic
    for m, *_ in cases[:2]:
        m.close()


def test_dot_noalloc_size_limit(sem):
    """At the stated maximum (2^27 local points: the 64^3 N=7 mesh) the result
    matches sem_dot; one more layer of elements is refused with a clear error,
    and the entry point works again afterwards."""
    import torch
    print_case("dot-noalloc-limit")
    bm = wl.box_mesh(64, N=7)
    assert bm.E * bm.Np == 2 ** 27
    m = sem.Mesh.from_box(bm)
    del bm
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    u = torch.rand((64 ** 3, 512), dtype=torch.float64, device="cuda", generator=g)
    v = torch.rand((64 ** 3, 512), dtype=torch.float64, device="cuda", generator=g)
    ref = sem.sem_dot(m.h, u, v)
    got = sem.sem_dot_noalloc(m.h, u, v)
    assert abs(got - ref) <= 1e-13 * ref
    m.close()
    del u, v
    bm = wl.box_mesh(64, 64, 65, N=7)
    m = sem.Mesh.from_box(bm)
    del bm
    u = torch.zeros((64 * 64 * 65, 512), dtype=torch.float64, device="cuda")
    with pytest.raises(sem.SemError, match="static scratch"):
        sem.sem_dot_noalloc(m.h, u, u)
    m.close()
    del u
    small = wl.box_mesh(2, N=3, deform=0.05, seed=9)
    ms, us, vs, ref, scale = _case(sem, small, 51, torch.float64)
    assert abs(sem.sem_dot_noalloc(ms.h, us, vs) - ref) <= 1e-13 * scale
    ms.close()

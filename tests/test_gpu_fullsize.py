"""Full-size checks in the configuration bench.py times.

64^3 elements, N=7 (134M local points): FP64 Ax on sampled elements against
the oracle (which recomputes those elements' geometric factors from their
coordinates), and the gather-scatter multiplicity histogram against the
lattice closed form. 48^3, N=7: the FP32-pMG flexible-CG solve reaches a true
residual <= 1e-8 and agrees with FP64 Jacobi-PCG."""
from math import comb

import numpy as np
import pytest

from oracle import operators as ops
from paper_2110_01716_amd import workloads as wl

from gpu_util import dev, host, print_case, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sem():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2110_01716_amd import sem as s
    s.load()
    return s


def test_ax_64cubed_sampled_elements(sem):
    import torch
    spec = wl.config_meshes()["ax_64x64x64_N7"]
    print_case("fullsize-ax", spec)
    bm = wl.box_mesh(spec["n"], N=spec["N"], deform=spec["deform"], seed=spec["seed"])
    m = sem.Mesh.from_box(bm)
    info = m.info()
    assert info["n_unique"] == (64 * 7 + 1) ** 3
    assert info["n_interior"] == (64 * 7 - 1) ** 3
    g = torch.Generator(device="cuda").manual_seed(7)
    u = torch.rand((bm.E, bm.Np), dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    Au = torch.empty_like(u)
    sem.sem_ax(m.h, u, Au)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.choice(bm.E, 120, replace=False), [0, bm.E - 1, 63, 64 * 64 - 1]]))
    it = torch.from_numpy(idx).to("cuda")
    us, As = host(u[it]), host(Au[it])
    G, _, _ = ops.geometric_factors(7, bm.x[idx], bm.y[idx], bm.z[idx])
    assert rel_err(As, ops.ax_local(7, G, us)) <= 1e-12
    # gather-scatter of ones: multiplicity histogram in closed form
    one = torch.ones_like(u)
    sem.sem_gs(m.h, one, apply_mask=False)
    vals, counts = torch.unique(one, return_counts=True)
    got = {int(v): int(c) for v, c in zip(vals.tolist(), counts.tolist())}
    n, N = 64, 7
    c2, c1 = n - 1, n * N + 1 - (n - 1)
    exp = {2 ** k: comb(3, k) * c2 ** k * c1 ** (3 - k) * 2 ** k for k in range(4)}
    assert got == exp
    del u, Au, one


def test_pmg_solve_48cubed(sem):
    import torch
    spec = wl.config_meshes()["pmg_48x48x48_N7"]
    print_case("fullsize-solve", spec)
    bm = wl.box_mesh(spec["n"], N=spec["N"], deform=spec["deform"], seed=spec["seed"])
    m = sem.Mesh.from_box(bm)
    p = sem.Pmg(m)
    assert p.info()["orders"] == [7, 3, 1]
    b = dev(wl.random_rhs(bm, 2000))
    x = torch.empty_like(b)
    info = sem.sem_pcg_solve(m.h, p.h, b, x, sem.solve_opts(rtol=1e-8))
    assert info["status"] == 0 and info["relres_true"] <= 1.05e-8 and info["iters"] <= 30
    # sampled Ax parity on this mesh (the operator whose residual was measured)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(bm.E, 60, replace=False))
    Ax = torch.empty_like(x)
    sem.sem_ax(m.h, x, Ax)
    it = torch.from_numpy(idx).to("cuda")
    G, _, _ = ops.geometric_factors(7, bm.x[idx], bm.y[idx], bm.z[idx])
    assert rel_err(host(Ax[it]), ops.ax_local(7, G, host(x[it]))) <= 1e-12
    # an independent algorithm reaches the same solution
    y = torch.empty_like(b)
    info2 = sem.sem_pcg_solve(m.h, None, b, y, sem.solve_opts(rtol=1e-10, maxit=20000))
    assert info2["status"] == 0
    assert float((x - y).abs().max() / y.abs().max()) <= 5e-6
    info3 = sem.sem_pcg_solve(m.h, p.h, b, x, sem.solve_opts(rtol=1e-11))
    assert info3["status"] == 0
    assert float((x - y).abs().max() / y.abs().max()) <= 1e-8

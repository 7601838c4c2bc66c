"""Full-size checks in the configuration bench.py times.

64^3 elements, N=7 (134M local points): FP64 Ax on sampled elements against
the oracle (which recomputes those elements' geometric factors from their
coordinates), and the gather-scatter multiplicity histogram against the
lattice closed form. 48^3, N=7: the FP32-pMG flexible-CG solve reaches a true
residual <= 1e-8, and at rtol 1e-10 it and FP64 Jacobi-PCG match the oracle's
x* to 1e-8 at 2000 sampled unique DOFs."""
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


def _oracle_samples(n):
    """x* of the oracle at seeded unique DOFs (tests/golden, written by
    make_oracle_solution_samples.py, which calls only the oracle)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        f"pmg_{n}x{n}x{n}_N7_rhs2000_xstar_samples.txt")
    meta, idx, val = {}, [], []
    for line in open(path):
        if line.startswith("#"):
            parts = line[1:].split()
            if len(parts) == 2:
                try:
                    meta[parts[0]] = float(parts[1])
                except ValueError:
                    pass
            continue
        i, v = line.split()
        idx.append(int(i))
        val.append(float(v))
    return meta, np.array(idx, dtype=np.int64), np.array(val)


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
    # the solution against the oracle's x* at 2000 sampled unique DOFs
    meta, sidx, sval = _oracle_samples(spec["n"])
    assert int(meta["n_unique"]) == m.info()["n_unique"]
    si = torch.from_numpy(sidx).to("cuda")

    def sampled_err(v):
        return float(np.max(np.abs(host(v.reshape(-1)[si]) - sval)) / meta["xstar_max_abs"])

    assert sampled_err(x) <= 1e-6
    info = sem.sem_pcg_solve(m.h, p.h, b, x, sem.solve_opts(rtol=1e-10))
    assert info["status"] == 0
    assert sampled_err(x) <= 1e-8
    # FP64 Jacobi-PCG reaches the same bar
    y = torch.empty_like(b)
    info2 = sem.sem_pcg_solve(m.h, None, b, y, sem.solve_opts(rtol=1e-10, maxit=20000))
    assert info2["status"] == 0
    assert sampled_err(y) <= 1e-8
    assert float((x - y).abs().max() / y.abs().max()) <= 1e-8

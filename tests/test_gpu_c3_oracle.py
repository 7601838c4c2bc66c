"""The mixed-precision solve against the FP64 oracle's solution, at a size that
runs the full-size code paths.

Mesh: the mixed-precision workload's construction (deformed box, N = 7, mesh
seed 1002, right-hand side seed 2000) at 16^3 elements: 2,097,152 local points,
enough for the vector kernels' multi-point-per-thread paths and for the
finalize kernel's multi-accumulator loop (more than 3072 block partials).

x* is the oracle's FP64 flexible CG with its FP64 p-multigrid V-cycle, solved
to relative residual 1e-12. Checks (relative max-norm error against x*):
  * FP32-pMG flexible CG (the paper's mixed-precision preconditioner) at
    rtol 1e-10 reaches a solution error <= 1e-8;
  * FP64 Jacobi-PCG at rtol 1e-10 reaches the same bar;
  * FlexCG iterates with the V-cycle in FP64, the oracle's rho per level and a
    fixed coarse iteration count equal the oracle's FlexCG iterates to 1e-10
    (the Polak-Ribiere recurrence step by step, including the GPU's
    rewritten numerator -alpha (z_new, w)).
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import pmg as opmg
from oracle import solvers
from paper_2110_01716_amd import workloads as wl

from gpu_util import dev, host, print_case, rel_err

# the oracle's setup and solve at this size take about a minute of host time
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

SIDE = 16


@pytest.fixture(scope="module")
def sem():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    from paper_2110_01716_amd import sem as s
    s.load()
    return s


@pytest.fixture(scope="module")
def problem():
    spec = wl.config_meshes()["pmg_48x48x48_N7"]
    bm = wl.box_mesh(SIDE, N=spec["N"], deform=spec["deform"], seed=spec["seed"])
    b = wl.random_rhs(bm, 2000)
    lv = opmg.build_levels(bm.N, bm.x, bm.y, bm.z, bm.gid, bm.dirichlet)
    return bm, b, lv


@pytest.fixture(scope="module")
def xstar(problem):
    bm, b, lv = problem
    res = opmg.pmg_flexcg(lv, b, opmg.VCycleOpts(), rtol=1e-12, maxit=60)
    assert res.relres <= 1e-12
    return res.x


@pytest.fixture(scope="module")
def mesh(sem, problem):
    bm, _, _ = problem
    m = sem.Mesh.from_box(bm)
    assert m.E * m.Np == SIDE ** 3 * 512
    return m


def test_fp32_pmg_flexcg_solution_vs_oracle(sem, problem, xstar, mesh):
    import torch
    bm, b, _ = problem
    print_case("c3-oracle-fp32-pmg", SIDE)
    p = sem.Pmg(mesh)
    assert p.info()["orders"] == [7, 3, 1]
    bd = dev(b)
    x = torch.empty_like(bd)
    errs = {}
    for rtol in (1e-8, 1e-10):
        info = sem.sem_pcg_solve(mesh.h, p.h, bd, x, sem.solve_opts(rtol=rtol))
        assert info["status"] == 0 and info["relres_true"] <= 1.05 * rtol
        errs[rtol] = rel_err(host(x), xstar)
    print("solution error vs oracle by rtol:", errs, flush=True)
    assert errs[1e-10] <= 1e-8
    assert errs[1e-8] <= 1e-6
    p.close()


def test_fp64_jacobi_pcg_solution_vs_oracle(sem, problem, xstar, mesh):
    import torch
    bm, b, _ = problem
    print_case("c3-oracle-jacobi-pcg", SIDE)
    bd = dev(b)
    x = torch.empty_like(bd)
    info = sem.sem_pcg_solve(mesh.h, None, bd, x, sem.solve_opts(rtol=1e-10, maxit=20000))
    assert info["status"] == 0 and info["relres_true"] <= 1.05e-10
    err = rel_err(host(x), xstar)
    print("Jacobi-PCG iterations", info["iters"], "error", err, flush=True)
    assert err <= 1e-8


def test_flexcg_fp64_pmg_iterates_match_oracle(sem, problem, mesh):
    import torch
    bm, b, lv = problem
    print_case("c3-oracle-flexcg-iterates", SIDE)
    G, _, _ = ops.geometric_factors(bm.N, bm.x, bm.y, bm.z)
    A = lambda v: ops.apply_A(bm.N, G, bm.gid, bm.dirichlet, v)  # noqa: E731
    dot = lambda u, v: ops.dot(bm.gid, u, v)  # noqa: E731
    fixed_coarse, iters = 6, 4
    p = sem.Pmg(mesh, smoother_dtype="f64", rho_override=[lv[0].rho, lv[1].rho], coarse_fixed_iters=fixed_coarse)
    bd = dev(b)
    x = torch.empty_like(bd)
    info = sem.sem_pcg_solve(mesh.h, p.h, bd, x, sem.solve_opts(fixed_iters=iters))
    o = opmg.VCycleOpts(coarse_fixed_iters=fixed_coarse)
    res = solvers.flexcg(A, lambda r: opmg.vcycle(lv, r, o), dot, b, fixed_iters=iters)
    assert info["status"] == 0 and info["iters"] == iters
    assert info["coarse_iters"] == iters * fixed_coarse
    assert rel_err(host(x), res.x) <= 1e-10
    assert abs(info["relres"] - res.relres) <= 1e-8 * res.relres
    p.close()


def test_dot_full_size(sem, problem, mesh):
    """Unique-DOF dot products over 2.1M points (the multi-point vector path)."""
    import torch
    bm, b, _ = problem
    print_case("c3-oracle-dot", SIDE)
    u = wl.random_rhs(bm, 11)  # consistent: every copy of an ID holds one value
    v = wl.random_rhs(bm, 12)
    got = sem.sem_dot(mesh.h, dev(u), dev(v))
    exp = ops.dot(bm.gid, u, v)
    scale = ops.dot(bm.gid, np.abs(u), np.abs(v))
    assert abs(got - exp) <= 1e-13 * scale

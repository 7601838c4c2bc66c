"""Projection onto prior solutions on the GPU against the oracle.

A sequence of smoothly varying right-hand sides is solved with the projected
starting guess. With a fixed number of inner iterations both sides take the
same steps, so the solutions and the basis (p_i and A p_i) are compared
element by element after every solve. Further cases: converged inner solves
against direct solves, a right-hand side in the span (no iterations), the
restart at L_max, iteration reduction with the pMG-preconditioned solver,
b = 0 and the error paths."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import projection as proj
from oracle import solvers
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


def _oracle(bm):
    N = bm.N
    G, B, _ = ops.geometric_factors(N, bm.x, bm.y, bm.z)
    A = lambda v: ops.apply_A(N, G, bm.gid, bm.dirichlet, v)  # noqa: E731
    dot = lambda a, b: ops.dot(bm.gid, a, b)  # noqa: E731
    Asp, ids, _ = ops.assemble(N, G, bm.gid, bm.dirichlet)
    lu = spla.splu(Asp.tocsc())
    idsall = np.unique(bm.gid)

    def direct(r, rtol=None):
        _, ru = ops.to_unique(bm.gid, r)
        return ops.scatter_unique(bm.gid, ids, lu.solve(ru[np.searchsorted(idsall, ids)]))

    dinv = ops.jacobi_inverse(N, G, bm.gid, bm.dirichlet)
    return A, dot, direct, dinv


def _basis(sem, pr, bm):
    import torch
    P, AP = [], []
    for i in range(pr.size):
        p = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        ap = torch.empty_like(p)
        pr.export(i, p, ap)
        P.append(host(p))
        AP.append(host(ap))
    return P, AP


def test_projection_fixed_iterations_match_oracle(sem):
    import torch
    print_case("proj-fixed-iters")
    bm = wl.box_mesh(3, 3, 2, N=5, deform=0.05, seed=31)
    A, dot, _, dinv = _oracle(bm)
    m = sem.Mesh.from_box(bm)
    pr = sem.Projection(m, L_max=8)
    sp = proj.ProjectionSpace(L_max=8)
    k = 12

    def inner(r, rtol):
        return solvers.pcg(A, lambda v: dinv * v, dot, r, fixed_iters=k).x

    seq = wl.rhs_sequence(bm, 6, modes=3, noise=1e-2, seed=7)
    for step, b in enumerate(seq):
        x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        info = pr.solve(None, dev(b), x, sem.solve_opts(rtol=1e-14, fixed_iters=k))
        xo, _, rel0 = proj.solve_projected(sp, A, dot, inner, b, rtol=1e-14)
        assert info["status"] == 0 and info["iters"] == k
        assert pr.size == sp.L == step + 1
        assert abs(info["relres_initial"] - rel0) <= 1e-9 * rel0
        assert rel_err(host(x), xo) <= 1e-10
    P, AP = _basis(sem, pr, bm)
    for i in range(sp.L):
        assert rel_err(P[i], sp.P[i]) <= 1e-9
        assert rel_err(AP[i], A(sp.P[i])) <= 1e-9
    M = np.array([[dot(p, A(q)) for q in P] for p in P])
    assert np.max(np.abs(M - np.eye(len(P)))) <= 1e-10


def test_projection_converged_solves_match_direct(sem):
    import torch
    print_case("proj-converged")
    bm = wl.box_mesh(4, 3, 3, N=4, deform=0.05, seed=32)
    A, dot, direct, _ = _oracle(bm)
    m = sem.Mesh.from_box(bm)
    pr = sem.Projection(m, L_max=10)
    sp = proj.ProjectionSpace(L_max=10)
    for b in wl.rhs_sequence(bm, 5, modes=4, noise=1e-3, seed=8):
        x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        info = pr.solve(None, dev(b), x, sem.solve_opts(rtol=1e-12))
        _, _, rel0 = proj.solve_projected(sp, A, dot, direct, b, rtol=1e-12)
        assert info["status"] == 0 and info["relres_true"] <= 2e-12
        assert abs(info["relres_initial"] - rel0) <= 1e-6 * rel0
        assert rel_err(host(x), direct(b)) <= 1e-9


def test_projection_rhs_in_span(sem):
    import torch
    print_case("proj-in-span")
    bm = wl.box_mesh(3, N=5, deform=0.05, seed=33)
    _, _, direct, _ = _oracle(bm)
    m = sem.Mesh.from_box(bm)
    pr = sem.Projection(m, L_max=10)
    seq = wl.rhs_sequence(bm, 3, modes=3, noise=1e-1, seed=9)
    for b in seq:
        x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        pr.solve(None, dev(b), x, sem.solve_opts(rtol=1e-13))
    b = 0.3 * seq[0] - 2.0 * seq[1] + seq[2]
    x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
    info = pr.solve(None, dev(b), x, sem.solve_opts(rtol=1e-9))
    assert info["status"] == 0 and info["iters"] == 0
    assert info["relres_initial"] <= 1e-10
    assert pr.size == 3
    assert rel_err(host(x), direct(b)) <= 1e-9


def test_projection_restart(sem):
    import torch
    print_case("proj-restart")
    bm = wl.box_mesh(3, N=4, deform=0.05, seed=34)
    A, dot, direct, _ = _oracle(bm)
    m = sem.Mesh.from_box(bm)
    pr = sem.Projection(m, L_max=3)
    sp = proj.ProjectionSpace(L_max=3)
    for k, b in enumerate(wl.rhs_sequence(bm, 5, modes=6, noise=1e-1, seed=10)):
        x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        pr.solve(None, dev(b), x, sem.solve_opts(rtol=1e-13))
        proj.solve_projected(sp, A, dot, direct, b, rtol=1e-13)
        assert pr.size == sp.L
    assert pr.size == 2  # restarted at the fourth solve, then grew by one
    P, AP = _basis(sem, pr, bm)
    for i in range(2):
        assert rel_err(P[i], sp.P[i]) <= 1e-8
        assert rel_err(AP[i], A(sp.P[i])) <= 1e-8


def test_projection_pmg_reduces_iterations(sem):
    import torch
    print_case("proj-pmg")
    bm = wl.box_mesh(4, N=7, deform=0.05, seed=35)
    m = sem.Mesh.from_box(bm)
    pmg = sem.Pmg(m)
    pr = sem.Projection(m, L_max=30)
    its, rel = [], []
    for b in wl.rhs_sequence(bm, 12, modes=4, noise=1e-6, seed=11):
        x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        info = pr.solve(pmg, dev(b), x, sem.solve_opts(rtol=1e-8))
        assert info["status"] == 0 and info["relres_true"] <= 1.5e-8
        its.append(info["iters"])
        rel.append(info["relres_initial"])
    assert rel[0] == 1.0
    assert max(rel[6:]) <= 1e-3
    assert max(its[6:]) < its[0]
    assert pr.size == 12 - its.count(0)


def test_projection_zero_rhs_and_errors(sem):
    import torch
    print_case("proj-errors")
    bm = wl.box_mesh(2, N=3)
    m = sem.Mesh.from_box(bm)
    pr = sem.Projection(m, L_max=4)
    b = torch.zeros(bm.x.shape, dtype=torch.float64, device="cuda")
    x = torch.full_like(b, 5.0)
    info = pr.solve(None, b, x)
    assert info["status"] == 0 and info["iters"] == 0 and pr.size == 0
    assert not torch.any(x != 0)
    info = pr.solve(None, b, x, sem.solve_opts(lam=1.0), check=False)
    assert info["rc"] == sem.SEM_EINVAL
    other = sem.Mesh.from_box(wl.box_mesh(2, N=3))
    pmg = sem.Pmg(other)
    info = pr.solve(pmg, b, x, check=False)
    assert info["rc"] == sem.SEM_EINVAL
    with pytest.raises(sem.SemError):
        sem.Projection(m, L_max=0)
    with pytest.raises(sem.SemError):
        pr.export(0, x)


def test_projection_with_gmres_matches_oracle(sem):
    import torch
    print_case("proj-gmres")
    bm = wl.box_mesh(3, 2, 3, N=5, deform=0.05, seed=36)
    A, dot, _, dinv = _oracle(bm)
    m = sem.Mesh.from_box(bm)
    pr = sem.Projection(m, L_max=6, gmres_K=4)
    sp = proj.ProjectionSpace(L_max=6)
    k = 7

    def inner(r, rtol):
        return solvers.fgmres(A, lambda v: dinv * v, dot, r, K=4, fixed_iters=k).x

    for step, b in enumerate(wl.rhs_sequence(bm, 4, modes=3, noise=1e-2, seed=12)):
        x = torch.empty(bm.x.shape, dtype=torch.float64, device="cuda")
        info = pr.solve(None, dev(b), x, sem.solve_opts(rtol=1e-14, fixed_iters=k))
        xo, _, rel0 = proj.solve_projected(sp, A, dot, inner, b, rtol=1e-14)
        assert info["status"] == 0 and info["iters"] == k and pr.size == sp.L
        assert abs(info["relres_initial"] - rel0) <= 1e-9 * rel0
        assert rel_err(host(x), xo) <= 1e-10
    P, AP = _basis(sem, pr, bm)
    for i in range(sp.L):
        assert rel_err(P[i], sp.P[i]) <= 1e-9

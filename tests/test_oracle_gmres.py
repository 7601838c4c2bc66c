"""Pins of the oracle's flexible GMRES.

What linear algebra fixes: the residual after j steps is the minimum of
|b - A x| over the right-preconditioned Krylov space (brute force over an
explicitly built basis); with the Jacobi preconditioner that space is the
one PCG searches, so GMRES's residual never exceeds PCG's; with a
preconditioner that changes between applications the flexible update keeps
the least-squares residual equal to the true one; a restarted solve reaches
the direct solution.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import solvers
from paper_2110_01716_amd import workloads as wl


def _setup(n=3, N=3, seed=12):
    m = wl.box_mesh(n, N=N, deform=0.05, seed=seed)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    mult = ops.multiplicity(m.gid)
    A = lambda v: ops.apply_A(N, G, m.gid, m.dirichlet, v)  # noqa: E731
    dot = lambda a, b: float(np.sum(a * b / mult))  # noqa: E731
    dinv = ops.jacobi_inverse(N, G, m.gid, m.dirichlet)
    return m, G, A, dot, dinv, mult


def test_residual_is_minimal_over_krylov_space():
    m, G, A, dot, dinv, mult = _setup()
    b = wl.random_rhs(m, 1)
    M = lambda v: dinv * v  # noqa: E731
    res = solvers.fgmres(A, M, dot, b, K=6, fixed_iters=6)
    wsq = np.sqrt(1.0 / mult).ravel()  # E-vector -> Euclidean over unique DOFs
    k = b / np.sqrt(dot(b, b))
    cols = []
    for j in range(6):
        c = M(k)
        cols.append(c)
        k = A(c)
        k = k / np.sqrt(dot(k, k))
        AC = np.stack([(A(c_) .ravel() * wsq) for c_ in cols], axis=1)
        y, *_ = np.linalg.lstsq(AC, b.ravel() * wsq, rcond=None)
        rmin = np.linalg.norm(b.ravel() * wsq - AC @ y) / np.sqrt(dot(b, b))
        assert abs(res.history[j] - rmin) <= 1e-6 * rmin


def test_gmres_residual_not_above_pcg():
    m, G, A, dot, dinv, _ = _setup(3, 4)
    b = wl.random_rhs(m, 2)
    M = lambda v: dinv * v  # noqa: E731
    g = solvers.fgmres(A, M, dot, b, K=20, fixed_iters=20)
    p = solvers.pcg(A, M, dot, b, fixed_iters=20)
    assert np.all(np.array(g.history) <= np.array(p.history) * (1 + 1e-9))


def test_flexible_update_with_varying_preconditioner():
    m, G, A, dot, dinv, _ = _setup()
    b = wl.random_rhs(m, 3)
    rng = np.random.default_rng(0)

    def M(v):  # a different (still SPD) scaling at every application
        return dinv * v * rng.uniform(0.5, 2.0) * (1.0 + 0.3 * np.cos(np.arange(v.size)).reshape(v.shape) ** 2)

    res = solvers.fgmres(A, M, dot, b, K=8, fixed_iters=8)
    r = b - A(res.x)
    true = np.sqrt(dot(r, r) / dot(b, b))
    assert abs(true - res.relres) <= 1e-9 * max(true, 1e-14) + 1e-13


def test_restarted_solve_reaches_direct_solution():
    m, G, A, dot, dinv, _ = _setup(3, 4)
    b = wl.random_rhs(m, 4)
    res = solvers.fgmres(A, lambda v: dinv * v, dot, b, K=3, rtol=1e-12, maxit=2000)
    Asp, ids, _ = ops.assemble(4, G, m.gid, m.dirichlet)
    idsall, bu = ops.to_unique(m.gid, b)
    x = ops.scatter_unique(m.gid, ids, spla.spsolve(Asp.tocsc(), bu[np.searchsorted(idsall, ids)]))
    assert res.relres <= 1e-12
    assert np.max(np.abs(res.x - x)) <= 1e-9 * np.max(np.abs(x))

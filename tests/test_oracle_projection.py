"""Pins of the oracle's projection onto prior solutions.

Checked against what linear algebra fixes, with exact (direct sparse) inner
solves: the basis is A-orthonormal; the best fit equals the A-orthogonal
projection onto the span of the raw earlier solutions computed from normal
equations; a right-hand side in the span of earlier ones is solved exactly by
projection alone; the restart keeps the newest solution; the projected solve
returns the solution of A x = b.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import projection as proj
from oracle import solvers
from paper_2110_01716_amd import workloads as wl


def _setup(n=3, N=3, seed=11):
    m = wl.box_mesh(n, N=N, deform=0.05, seed=seed)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    mult = ops.multiplicity(m.gid)
    A = lambda v: ops.apply_A(N, G, m.gid, m.dirichlet, v)  # noqa: E731
    dot = lambda a, b: float(np.sum(a * b / mult))  # noqa: E731
    Asp, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    lu = spla.splu(Asp.tocsc())
    idsall = np.unique(m.gid)

    def direct(r, rtol=None):
        _, ru = ops.to_unique(m.gid, r)
        return ops.scatter_unique(m.gid, ids, lu.solve(ru[np.searchsorted(idsall, ids)]))

    dinv = ops.jacobi_inverse(N, G, m.gid, m.dirichlet)
    return m, A, dot, direct, dinv


def test_basis_is_A_orthonormal():
    m, A, dot, direct, _ = _setup()
    seq = wl.rhs_sequence(m, 8, modes=4, noise=1e-2, seed=1)
    sp = proj.ProjectionSpace(L_max=10)
    for b in seq:
        proj.solve_projected(sp, A, dot, direct, b, rtol=1e-12)
    assert sp.L == 8
    M = np.array([[dot(p, A(q)) for q in sp.P] for p in sp.P])
    assert np.max(np.abs(M - np.eye(sp.L))) <= 1e-10


def test_best_fit_is_A_orthogonal_projection():
    """xbar = argmin over span(x_1..x_L) of |x - A^-1 b|_A, from normal equations."""
    m, A, dot, direct, _ = _setup()
    seq = wl.rhs_sequence(m, 6, modes=3, noise=5e-2, seed=2)
    sp = proj.ProjectionSpace(L_max=10)
    X = []
    for b in seq[:5]:
        x, _, _ = proj.solve_projected(sp, A, dot, direct, b, rtol=1e-13)
        X.append(x)
    b = seq[5]
    gram = np.array([[dot(xi, A(xj)) for xj in X] for xi in X])
    rhs = np.array([dot(xi, b) for xi in X])
    c = np.linalg.solve(gram, rhs)
    xstar = sum(ci * xi for ci, xi in zip(c, X))
    xbar = proj.best_fit(sp, dot, b)
    assert np.max(np.abs(xbar - xstar)) <= 1e-9 * np.max(np.abs(xstar))
    # the fit's error is A-orthogonal to every earlier solution
    e = direct(b) - xbar
    for xi in X:
        assert abs(dot(xi, A(e))) <= 1e-9 * np.sqrt(dot(xi, A(xi)) * dot(e, A(e)))


def test_rhs_in_span_is_solved_by_projection():
    m, A, dot, direct, _ = _setup()
    seq = wl.rhs_sequence(m, 3, modes=3, noise=1e-1, seed=3)
    sp = proj.ProjectionSpace(L_max=10)
    for b in seq:
        proj.solve_projected(sp, A, dot, direct, b, rtol=1e-13)
    b = 0.3 * seq[0] - 2.0 * seq[1] + seq[2]
    x, dx, rel0 = proj.solve_projected(sp, A, dot, direct, b, rtol=1e-9)
    assert rel0 <= 1e-10
    assert not np.any(dx)
    assert sp.L == 3  # nothing added
    xd = direct(b)
    assert np.max(np.abs(x - xd)) <= 1e-9 * np.max(np.abs(xd))


def test_projected_solve_returns_the_solution():
    m, A, dot, direct, _ = _setup()
    seq = wl.rhs_sequence(m, 5, modes=6, noise=1e-2, seed=4)
    sp = proj.ProjectionSpace(L_max=10)
    for b in seq:
        x, _, rel0 = proj.solve_projected(sp, A, dot, direct, b, rtol=1e-12)
        xd = direct(b)
        assert np.max(np.abs(x - xd)) <= 1e-9 * np.max(np.abs(xd))


def test_restart_keeps_newest_solution():
    m, A, dot, direct, _ = _setup()
    seq = wl.rhs_sequence(m, 4, modes=6, noise=1e-1, seed=5)
    sp = proj.ProjectionSpace(L_max=3)
    for k, b in enumerate(seq):
        x, _, _ = proj.solve_projected(sp, A, dot, direct, b, rtol=1e-12)
        assert sp.L == (k + 1 if k < 3 else 1)
    p = sp.P[0]
    assert abs(dot(p, A(p)) - 1.0) <= 1e-12
    s = dot(p, x) / dot(p, p)
    assert np.max(np.abs(s * p - x)) <= 1e-12 * np.max(np.abs(x))


def test_projection_shrinks_residual_for_smooth_sequence():
    """With an iterative inner solve: the projected residual drops to the
    noise level once the space spans the smooth modes, iterations drop, and
    the final residual meets the tolerance relative to |b|."""
    m, A, dot, _, dinv = _setup(3, 4)
    seq = wl.rhs_sequence(m, 10, modes=3, noise=1e-4, seed=6)
    sp = proj.ProjectionSpace(L_max=30)
    its = []

    def inner(r, rtol):
        res = solvers.pcg(A, lambda v: dinv * v, dot, r, rtol=rtol)
        its.append(res.iters)
        return res.x

    rel = []
    for b in seq:
        x, _, rel0 = proj.solve_projected(sp, A, dot, inner, b, rtol=1e-8)
        rel.append(rel0)
        r = b - A(x)
        assert np.sqrt(dot(r, r)) <= 1.5e-8 * np.sqrt(dot(b, b))
    assert rel[0] == 1.0
    assert max(rel[4:]) <= 1e-3
    assert its[-1] < its[0]

"""Pins of the oracle's solvers, smoother, transfers and V-cycle.

Library routines (a direct sparse solve, a sparse eigensolver), closed forms
(the Chebyshev error polynomial), exact-arithmetic identities (flexible CG
with a fixed preconditioner equals PCG; restriction is the adjoint of
prolongation; prolongation reproduces coarse polynomials) and structural
properties (a symmetric V-cycle with an exact coarse solve).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import pmg, solvers
from oracle.counter_rng import start_vector
from paper_2110_01716_amd import workloads as wl


def _setup(n=2, N=4, deform=0.05, seed=5):
    m = wl.box_mesh(n, N=N, deform=deform, seed=seed)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    mult = ops.multiplicity(m.gid)
    A = lambda v: ops.apply_A(N, G, m.gid, m.dirichlet, v)  # noqa: E731
    dot = lambda a, b: float(np.sum(a * b / mult))  # noqa: E731
    dinv = ops.jacobi_inverse(N, G, m.gid, m.dirichlet)
    return m, G, B, A, dot, dinv


def _direct(m, N, G, b):
    Asp, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    idsall, bu = ops.to_unique(m.gid, b)
    xin = spla.spsolve(Asp.tocsc(), bu[np.searchsorted(idsall, ids)])
    return ops.scatter_unique(m.gid, ids, xin)


def test_pcg_matches_direct_solve():
    N = 4
    m, G, B, A, dot, dinv = _setup(3, N)
    b = wl.random_rhs(m, 1)
    res = solvers.pcg(A, lambda r: dinv * r, dot, b, rtol=1e-13)
    x = _direct(m, N, G, b)
    assert np.max(np.abs(res.x - x)) <= 1e-10 * np.max(np.abs(x))
    assert res.relres <= 1e-13
    # the recurrence residual equals the true residual to rounding
    assert np.sqrt(dot(b - A(res.x), b - A(res.x))) <= 1e-12 * np.sqrt(dot(b, b))


def test_flexcg_equals_pcg_with_fixed_preconditioner():
    N = 3
    m, G, B, A, dot, dinv = _setup(3, N)
    b = wl.random_rhs(m, 2)
    M = lambda r: dinv * r  # noqa: E731
    a = solvers.pcg(A, M, dot, b, fixed_iters=12)
    f = solvers.flexcg(A, M, dot, b, fixed_iters=12)
    np.testing.assert_allclose(np.array(f.history), np.array(a.history), rtol=1e-8)
    assert np.max(np.abs(a.x - f.x)) <= 1e-8 * np.max(np.abs(a.x))


def test_pcg_zero_rhs():
    m, G, B, A, dot, dinv = _setup(2, 2)
    res = solvers.pcg(A, lambda r: dinv * r, dot, np.zeros_like(m.x))
    assert res.iters == 0 and np.all(res.x == 0)


@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_chebyshev_error_polynomial(degree):
    # diagonal SPD operator with known spectrum, D = I: after one sweep from 0,
    # e_k = T_k((theta - l)/delta) / T_k(theta/delta) e_0 per eigencomponent
    lam = np.linspace(0.05, 2.0, 37)
    x_true = np.random.default_rng(degree).standard_normal(lam.size)
    r = lam * x_true
    rho = lam.max()
    x = solvers.chebyshev(lambda v: lam * v, np.ones_like(lam), r, rho, degree, 0.1, 1.1)
    a, b = 0.1 * rho, 1.1 * rho
    th, de = (a + b) / 2, (b - a) / 2
    def Tk(k, t):
        t = np.asarray(t, dtype=float)
        out = np.empty_like(t)
        inside = np.abs(t) <= 1
        out[inside] = np.cos(k * np.arccos(t[inside]))
        out[~inside] = np.sign(t[~inside]) ** k * np.cosh(k * np.arccosh(np.abs(t[~inside])))
        return out
    pk = Tk(degree, (th - lam) / de) / Tk(degree, np.array([th / de]))[0]
    np.testing.assert_allclose(x_true - x, pk * x_true, atol=1e-12)


def test_chebyshev_restart_from_x0():
    lam = np.linspace(0.1, 1.0, 20)
    xt = np.arange(1.0, 21.0)
    r = lam * xt
    x1 = solvers.chebyshev(lambda v: lam * v, np.ones_like(lam), r, 1.0, 2)
    x2 = solvers.chebyshev(lambda v: lam * v, np.ones_like(lam), r, 1.0, 2, x0=x1)
    # two sweeps: error multiplies by p_2 twice
    e1, e2 = xt - x1, xt - x2
    np.testing.assert_allclose(e2, e1 * (e1 / xt), rtol=1e-9, atol=1e-12)


def test_power_iteration_vs_eigensolver():
    N = 4
    m, G, B, A, dot, dinv = _setup(3, N)
    Asp, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    d = Asp.diagonal()
    lmax = spla.eigsh(Asp, k=1, M=sp.diags(d), which="LA", return_eigenvectors=False)[0]
    v0 = ops.mask(m.dirichlet, start_vector(m.gid))
    rho = solvers.power_rho(A, dinv, dot, v0, iters=200)
    assert abs(rho - lmax) <= 2e-3 * lmax
    rho20 = solvers.power_rho(A, dinv, dot, v0, iters=20)
    assert 0.7 * lmax <= rho20 <= lmax * (1 + 1e-12)


@pytest.mark.parametrize("Nf,Nc", [(7, 3), (3, 1), (5, 2)])
def test_transfers_adjoint_and_exact(Nf, Nc):
    m = wl.box_mesh(2, N=Nf, deform=0.05, seed=6)
    levels = pmg.build_levels(Nf, m.x, m.y, m.z, m.gid, m.dirichlet, orders=[Nf, Nc] + ([1] if Nc > 1 else []),
                              rho=[1.0, 1.0])
    f, c = levels[0], levels[1]
    rng = np.random.default_rng(0)
    rf = ops.mask(f.dirichlet, ops.gs(f.gid, rng.standard_normal(f.x.shape)) / f.mult)
    vc = ops.mask(c.dirichlet, ops.gs(c.gid, rng.standard_normal(c.x.shape)) / c.mult)
    lhs = c.dot(pmg.restrict(levels, 0, rf), vc)
    rhs = f.dot(rf, pmg.prolong(levels, 0, vc))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-300) + 1e-14
    # prolongation of a consistent coarse field is consistent
    p = pmg.prolong(levels, 0, vc)
    np.testing.assert_allclose(ops.gs(f.gid, p / f.mult), p, atol=1e-13)
    # exact on the coarse map's polynomials: the coarse coordinate field is
    # reproduced at the fine points up to interpolation of the geometry
    ma = wl.box_mesh(2, N=Nf)
    la = pmg.build_levels(Nf, ma.x, ma.y, ma.z, ma.gid, ma.dirichlet, orders=[Nf, Nc] + ([1] if Nc > 1 else []),
                          rho=[1.0, 1.0])
    for deg in range(Nc + 1):
        np.testing.assert_allclose(pmg.prolong(la, 0, la[1].x ** deg), la[0].x ** deg, atol=1e-13)


def test_coarse_connectivity_matches_lattice():
    N = 7
    m = wl.box_mesh(3, N=N, deform=0.05, seed=8)
    levels = pmg.build_levels(N, m.x, m.y, m.z, m.gid, m.dirichlet, rho=[1.0, 1.0])
    for lev in levels[1:]:
        lat = wl.box_mesh(3, N=lev.N)  # lattice IDs and boundary flags at that order
        # same equivalence classes: a bijection between the two labelings
        pairs = np.unique(np.stack([lev.gid.ravel(), lat.gid.ravel()], 1), axis=0)
        assert len(pairs) == len(np.unique(lev.gid)) == len(np.unique(lat.gid)) == (3 * lev.N + 1) ** 3
        np.testing.assert_array_equal(lev.dirichlet, lat.dirichlet)


def test_coarse_geometry_affine_closed_form():
    m = wl.box_mesh(2, N=7)
    levels = pmg.build_levels(7, m.x, m.y, m.z, m.gid, m.dirichlet, rho=[1.0, 1.0])
    for lev in levels[1:]:
        a = wl.box_mesh(2, N=lev.N)
        np.testing.assert_allclose(lev.x, a.x, atol=1e-14)
        Ga, _, _ = ops.geometric_factors(lev.N, a.x, a.y, a.z)
        np.testing.assert_allclose(lev.G, Ga, rtol=1e-12, atol=1e-15)


def test_vcycle_symmetric_with_exact_coarse_solve():
    N = 5
    m = wl.box_mesh(2, N=N, deform=0.05, seed=9)
    levels = pmg.build_levels(N, m.x, m.y, m.z, m.gid, m.dirichlet, orders=[5, 2, 1])
    o = pmg.VCycleOpts(coarse_exact=True)
    top = levels[0]
    rng = np.random.default_rng(1)
    u = ops.mask(top.dirichlet, ops.gs(top.gid, rng.standard_normal(top.x.shape)) / top.mult)
    v = ops.mask(top.dirichlet, ops.gs(top.gid, rng.standard_normal(top.x.shape)) / top.mult)
    a = top.dot(v, pmg.vcycle(levels, u, o))
    b = top.dot(u, pmg.vcycle(levels, v, o))
    assert abs(a - b) <= 1e-11 * abs(a)
    # and it is a contraction: ||I - M A|| < 1 on a random error
    e = u
    for _ in range(3):
        e = e - pmg.vcycle(levels, top.A(e), o)
    assert np.sqrt(top.dot(e, top.A(e))) < 0.2 * np.sqrt(top.dot(u, top.A(u)))


def test_pmg_flexcg_solution_matches_direct():
    N = 5
    m = wl.box_mesh(2, N=N, deform=0.05, seed=12)
    levels = pmg.build_levels(N, m.x, m.y, m.z, m.gid, m.dirichlet)
    b = wl.random_rhs(m, 3)
    res = pmg.pmg_flexcg(levels, b, rtol=1e-12)
    x = _direct(m, N, levels[0].G, b)
    assert np.max(np.abs(res.x - x)) <= 1e-10 * np.max(np.abs(x))
    assert res.iters < 25


def _varying_preconditioner(dinv, seed=0):
    rng = np.random.default_rng(seed)

    def M(v):  # a different SPD scaling at every application
        wgt = 1.0 + 0.5 * np.cos(np.arange(v.size) * rng.uniform(0.1, 3.0)).reshape(v.shape) ** 2
        return dinv * v * wgt
    return M


def _local_a_orthogonality(flex, N=4, iters=10):
    """max_k |(p_{k+1}, A p_k)| / (|p_{k+1}|_A |p_k|_A) of a flexible-CG run."""
    m, G, B, A, dot, dinv = _setup(3, N)
    b = wl.random_rhs(m, 21)
    seen = []
    flex(A, _varying_preconditioner(dinv), dot, b, fixed_iters=iters,
         callback=lambda k, p, w: seen.append((p.copy(), w.copy())))
    cos = []
    for (p0, w0), (p1, w1) in zip(seen, seen[1:]):
        cos.append(abs(dot(p1, w0)) / np.sqrt(dot(p0, w0) * dot(p1, w1)))
    return max(cos)


def test_flexcg_polak_ribiere_keeps_local_a_orthogonality():
    # With beta = (z_new, r_new - r_old) / (z_old, r_old) and r_new - r_old =
    # -alpha A p_k, beta equals -(z_new, A p_k) / (p_k, A p_k): the new search
    # direction is A-orthogonal to the previous one whatever the
    # preconditioner did (Notay 2000). Fletcher-Reeves' (z_new, r_new) /
    # (z_old, r_old) equals it only when M is fixed.
    assert _local_a_orthogonality(solvers.flexcg) <= 1e-10


def test_local_a_orthogonality_rejects_fletcher_reeves():
    # the same check on a copy of the oracle's flexible CG with the
    # Fletcher-Reeves beta planted in it must fail
    import inspect
    src = inspect.getsource(solvers.flexcg)
    assert "dot(z, r - r_old) / rz" in src
    ns = dict(solvers.__dict__)
    exec(compile(src.replace("dot(z, r - r_old) / rz", "dot(z, r) / rz"), "<mutated flexcg>", "exec"), ns)
    assert _local_a_orthogonality(ns["flexcg"]) > 1e-3

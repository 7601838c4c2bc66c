"""Pins of the oracle's Helmholtz operator (A + lambda B), the velocity-substep
operator solved by Jacobi-PCG: positive definite without Dirichlet conditions,
exact diagonal, and spectral convergence of a manufactured Neumann solution."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import solvers
from paper_2110_01716_amd import workloads as wl


@pytest.mark.parametrize("lam", [0.5, 10.0])
def test_neumann_helmholtz_is_spd(lam):
    N = 3
    m = wl.box_mesh(2, N=N, deform=0.05, seed=3, dirichlet=False)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    H, _ = ops.assemble_helmholtz(N, G, B, lam, m.gid, m.dirichlet)
    Hd = H.toarray()
    np.testing.assert_allclose(Hd, Hd.T, atol=1e-13 * np.abs(Hd).max())
    np.linalg.cholesky(Hd)
    # the constant mode: (1, H 1) = lam * volume
    one = np.ones(Hd.shape[0])
    vol = float(np.sum(B))
    assert abs(one @ Hd @ one - lam * vol) <= 1e-11 * lam * vol


def test_helmholtz_diagonal_vs_assembled():
    N, lam = 4, 3.0
    m = wl.box_mesh(2, N=N, deform=0.05, seed=5)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    H, ids = ops.assemble_helmholtz(N, G, B, lam, m.gid, m.dirichlet)
    dinv = ops.helmholtz_jacobi_inverse(N, G, B, lam, m.gid, m.dirichlet)
    idsall, du = ops.to_unique(m.gid, dinv)
    np.testing.assert_allclose(du[np.searchsorted(idsall, ids)], 1.0 / H.diagonal(), rtol=1e-12)


def _neumann_error(N, lam=2.0, n=2):
    m = wl.box_mesh(n, N=N, dirichlet=False)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    u = wl.manufactured_neumann_solution(m)
    f = (3 * np.pi ** 2 + lam) * u
    b = ops.gs(m.gid, B * f)
    H, ids = ops.assemble_helmholtz(N, G, B, lam, m.gid, m.dirichlet)
    idsall, bu = ops.to_unique(m.gid, b)
    x = ops.scatter_unique(m.gid, ids, spla.spsolve(H.tocsc(), bu[np.searchsorted(idsall, ids)]))
    return np.max(np.abs(x - u))


def test_manufactured_neumann_spectral_convergence():
    errs = [_neumann_error(N) for N in range(2, 9)]
    for k in range(len(errs) - 2):
        assert errs[k + 2] < 0.2 * errs[k], errs
    assert errs[-1] < 1e-6, errs


def test_helmholtz_pcg_matches_direct():
    N, lam = 4, 7.0
    m = wl.box_mesh(3, N=N, deform=0.05, seed=9)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    b = wl.random_rhs(m, 3)
    dinv = ops.helmholtz_jacobi_inverse(N, G, B, lam, m.gid, m.dirichlet)
    res = solvers.pcg(lambda v: ops.apply_H(N, G, B, lam, m.gid, m.dirichlet, v), lambda r: dinv * r,
                      lambda a, c: ops.dot(m.gid, a, c), b, rtol=1e-13)
    H, ids = ops.assemble_helmholtz(N, G, B, lam, m.gid, m.dirichlet)
    idsall, bu = ops.to_unique(m.gid, b)
    x = ops.scatter_unique(m.gid, ids, spla.spsolve(H.tocsc(), bu[np.searchsorted(idsall, ids)]))
    assert np.max(np.abs(res.x - x)) <= 1e-10 * np.max(np.abs(x))

"""Pins of the oracle's SEM operators: geometry, Ax, gather-scatter, diagonal.

Closed forms (affine elements), the exact weak form on polynomials, null space,
symmetry, positive definiteness, the continuous spectrum and spectral
convergence of a manufactured solution: each would fail on a dropped term, a
wrong sign or index, or a transposed operand somewhere in the oracle.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import operators as ops
from oracle import reference_ops as ro
from paper_2110_01716_amd import workloads as wl


def _rng(s):
    return np.random.default_rng(s)


@pytest.mark.parametrize("N", [1, 3, 5, 7])
def test_affine_geometric_factors(N):
    n = 3
    m = wl.box_mesh(n, N=N)
    G, B, detJ = ops.geometric_factors(N, m.x, m.y, m.z)
    h = 1.0 / n
    _, w = ro.gll(N)
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    np.testing.assert_allclose(detJ, h ** 3 / 8, rtol=1e-12)
    for s, name in enumerate(ops.G_NAMES):
        if name in ("rr", "ss", "tt"):
            np.testing.assert_allclose(G[:, s], np.broadcast_to(W * h / 2, G[:, s].shape), rtol=1e-12)
        else:
            assert np.max(np.abs(G[:, s])) < 1e-13 * np.max(np.abs(G[:, 0]))
    np.testing.assert_allclose(B.sum(), 1.0, rtol=1e-13)


def test_affine_box_anisotropic_geometry():
    # a brick of sides hx, hy, hz: G_rr = W hy hz / (2 hx), etc.
    N = 4
    m = wl.box_mesh(2, 3, 4, N=N, hi=(2.0, 3.0, 1.0))
    hx, hy, hz = 1.0, 1.0, 0.25
    G, B, detJ = ops.geometric_factors(N, m.x, m.y, m.z)
    _, w = ro.gll(N)
    W = np.einsum("k,j,i->kji", w, w, w).ravel()
    np.testing.assert_allclose(G[:, 0], np.broadcast_to(W * hy * hz / (2 * hx), G[:, 0].shape), rtol=1e-12)
    np.testing.assert_allclose(G[:, 3], np.broadcast_to(W * hx * hz / (2 * hy), G[:, 3].shape), rtol=1e-12)
    np.testing.assert_allclose(G[:, 5], np.broadcast_to(W * hx * hy / (2 * hz), G[:, 5].shape), rtol=1e-12)
    np.testing.assert_allclose(B.sum(), 6.0, rtol=1e-13)


@pytest.mark.parametrize("N", [2, 4, 7])
def test_ax_affine_kronecker_closed_form(N):
    # A^e = (h/2)(Bh x Bh x Ah + Bh x Ah x Bh + Ah x Bh x Bh), Ah = D^T Bh D
    n = 2
    m = wl.box_mesh(n, N=N)
    G, _, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    D = ro.deriv_matrix(N)
    _, w = ro.gll(N)
    Bh = np.diag(w)
    Ah = D.T @ Bh @ D
    h = 1.0 / n
    Ae = (h / 2) * (np.kron(Bh, np.kron(Bh, Ah)) + np.kron(Bh, np.kron(Ah, Bh))
                    + np.kron(Ah, np.kron(Bh, Bh)))
    u = _rng(N).standard_normal(m.x.shape)
    ref = u @ Ae.T
    got = ops.ax_local(N, G, u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [3, 7])
def test_ax_matrix_free_vs_element_matrices(N):
    m = wl.box_mesh(2, N=N, deform=0.05, seed=3)
    G, _, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    Ae = ops.element_matrices(N, G)
    u = _rng(1).standard_normal(m.x.shape)
    ref = np.einsum("epq,eq->ep", Ae, u)
    got = ops.ax_local(N, G, u)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("N", [2, 5, 7])
def test_ax_null_space_and_symmetry(N):
    m = wl.box_mesh(3, N=N, deform=0.05, seed=7, dirichlet=False)
    G, _, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    one = np.ones_like(m.x)
    A1 = ops.ax_local(N, G, one)
    scale = np.max(np.abs(G))
    assert np.max(np.abs(A1)) <= 1e-12 * scale * N * N
    u = ops.gs(m.gid, _rng(2).standard_normal(m.x.shape)) / ops.multiplicity(m.gid)
    v = ops.gs(m.gid, _rng(3).standard_normal(m.x.shape)) / ops.multiplicity(m.gid)
    Au = ops.apply_A(N, G, m.gid, m.dirichlet, u)
    Av = ops.apply_A(N, G, m.gid, m.dirichlet, v)
    a, b = ops.dot(m.gid, v, Au), ops.dot(m.gid, u, Av)
    assert abs(a - b) <= 1e-13 * abs(a)


@pytest.mark.parametrize("N", [2, 3, 4])
def test_spd_under_dirichlet(N):
    m = wl.box_mesh(2, N=N, deform=0.05, seed=11)
    G, _, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    A, _, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    Ad = A.toarray()
    np.testing.assert_allclose(Ad, Ad.T, atol=1e-13 * np.abs(Ad).max())
    np.linalg.cholesky(Ad)
    assert np.linalg.eigvalsh(Ad).min() > 0


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (4, 4), (5, 2)])
def test_exact_bilinear_form(a, b):
    # affine mesh, u = x^a, v = x^b: v^T A u = a b int x^(a+b-2) dV = a b / (a+b-1)
    N = 5
    m = wl.box_mesh(3, N=N, dirichlet=False)
    G, _, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    u, v = m.x ** a, m.x ** b
    val = float(np.sum(v * ops.ax_local(N, G, u)))
    assert abs(val - a * b / (a + b - 1)) < 1e-12


def test_spectrum_lowest_eigenvalue():
    # Dirichlet Laplacian on the unit cube: lambda_min = 3 pi^2
    N = 6
    m = wl.box_mesh(2, N=N)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    A, _, Bd = ops.assemble(N, G, m.gid, m.dirichlet, B)
    import scipy.sparse as sp
    lam = spla.eigsh(A, k=1, M=sp.diags(Bd), sigma=0, which="LM", return_eigenvectors=False)
    assert abs(lam[0] - 3 * np.pi ** 2) < 1e-5 * 3 * np.pi ** 2


def _manufactured_error(N, n=2):
    m = wl.box_mesh(n, N=N)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    A, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    b = ops.assemble_rhs(N, B, m.gid, m.dirichlet, wl.manufactured_source(m))
    idsall, bu = ops.to_unique(m.gid, b)
    rhs = bu[np.searchsorted(idsall, ids)]
    xin = spla.spsolve(A.tocsc(), rhs)
    x = ops.scatter_unique(m.gid, ids, xin)
    return np.max(np.abs(x - wl.manufactured_solution(m)))


def test_manufactured_spectral_convergence():
    errs = [_manufactured_error(N) for N in range(2, 10)]
    # geometric decay in N until round-off
    for k in range(len(errs) - 2):
        assert errs[k + 2] < 0.2 * errs[k], errs
    assert errs[-1] < 1e-7, errs


def test_gather_scatter_properties():
    N = 4
    n = 3
    m = wl.box_mesh(n, N=N, deform=0.05, seed=2)
    mult = ops.gs(m.gid, np.ones_like(m.x))
    assert set(np.unique(mult)) == {1.0, 2.0, 4.0, 8.0}
    np.testing.assert_allclose(np.sum(1.0 / mult), (n * N + 1) ** 3, rtol=1e-13)
    c = ops.gs(m.gid, _rng(4).standard_normal(m.x.shape))  # consistent
    np.testing.assert_allclose(ops.gs(m.gid, c / mult), c, rtol=1e-13)
    # random relabelling and element permutation give the same result
    r = wl.relabel(m, 9)
    v = _rng(5).standard_normal(m.x.shape)
    np.testing.assert_allclose(ops.gs(r.gid, v[r.meta["perm"]]), ops.gs(m.gid, v)[r.meta["perm"]],
                               rtol=1e-14)


@pytest.mark.parametrize("N", [2, 4, 7])
def test_jacobi_diagonal_vs_assembled(N):
    m = wl.box_mesh(2, N=N, deform=0.05, seed=4)
    G, _, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    A, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    dinv = ops.jacobi_inverse(N, G, m.gid, m.dirichlet)
    idsall, du = ops.to_unique(m.gid, dinv)
    got = du[np.searchsorted(idsall, ids)]
    np.testing.assert_allclose(got, 1.0 / A.diagonal(), rtol=1e-12)
    assert np.all(dinv[m.dirichlet != 0] == 0)


def test_helmholtz_adds_mass():
    N = 3
    m = wl.box_mesh(2, N=N, deform=0.05, seed=4)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    u = _rng(8).standard_normal(m.x.shape)
    np.testing.assert_allclose(ops.helmholtz_local(N, G, B, 2.5, u) - ops.ax_local(N, G, u),
                               2.5 * B * u, rtol=1e-12, atol=1e-14)
    # B integrates x^2 exactly on an affine mesh: sum B x^2 = 1/3
    ma = wl.box_mesh(2, N=N)
    _, Ba, _ = ops.geometric_factors(N, ma.x, ma.y, ma.z)
    assert abs(np.sum(Ba * ma.x ** 2) - 1 / 3) < 1e-14


def _linear_field_forms(N, m, G):
    """[E, 3, 3]: x_a^T A^e x_b per element for the coordinate fields x, y, z."""
    X = (m.x, m.y, m.z)
    AX = [ops.ax_local(N, G, c) for c in X]
    return np.stack([np.stack([np.sum(X[a] * AX[b], axis=1) for b in range(3)], axis=1) for a in range(3)],
                    axis=1)


@pytest.mark.parametrize("N", [2, 5, 7])
def test_linear_fields_on_deformed_mesh(N):
    # The coordinate fields x_a are exactly in the isoparametric space, so the
    # discrete gradient of x_a is the unit vector e_a at every quadrature point
    # and the weak form gives x_a^T A^e x_b = delta_ab * sum_p B_p on every
    # element, for any (non-affine) deformation. A geometric factor built from
    # a transposed inverse Jacobian, a swapped pair of G slots or a wrong
    # weight breaks it.
    m = wl.box_mesh(3, N=N, deform=0.05, seed=13, dirichlet=False)
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    F = _linear_field_forms(N, m, G)
    vol = B.sum(axis=1)
    for a in range(3):
        for b in range(3):
            want = vol if a == b else np.zeros_like(vol)
            assert np.max(np.abs(F[:, a, b] - want)) <= 1e-12 * vol.max(), (a, b)
    # the deformation is genuinely non-affine: J varies inside elements
    assert np.ptp(G[:, 1]) > 1e-3 * np.abs(G[:, 0]).max()


def test_linear_field_identity_rejects_transposed_inverse(monkeypatch):
    # a plausible mistake planted in the oracle (d r / d x read as the
    # transpose of the inverse Jacobian) must fail the identity above
    N = 5
    m = wl.box_mesh(3, N=N, deform=0.05, seed=13, dirichlet=False)
    inv = np.linalg.inv
    monkeypatch.setattr(np.linalg, "inv", lambda a: np.swapaxes(inv(a), -1, -2))
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    F = _linear_field_forms(N, m, G)
    vol = B.sum(axis=1)
    dev = max(np.max(np.abs(F[:, a, b] - (vol if a == b else 0.0))) for a in range(3) for b in range(3))
    assert dev > 1e-4 * vol.max()

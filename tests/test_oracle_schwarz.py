"""Pins of the oracle's overlapping Schwarz / fast-diagonalization smoother.

Checked against what the mathematics fixes, on undeformed (affine) bricks
where the separable local operator is exact: the extension's global IDs are
the lattice neighbours; the Kronecker operator built from the extended 1D
matrices equals the assembled SEM stiffness on the extended box; the fast
diagonalization solve equals a dense solve of that operator (interior and
boundary elements, Dirichlet and Neumann ends); a single Dirichlet brick is
solved exactly; the counting function matches lattice brute force; the
unweighted additive operator is symmetric.
"""
import numpy as np
import pytest

from oracle import operators as ops
from oracle import schwarz
from paper_2110_01716_amd import workloads as wl


def _kron_op(A1, B1):
    (Ar, Br), (As, Bs), (At, Bt) = zip(A1, B1)
    return (np.kron(Bt, np.kron(Bs, Ar)) + np.kron(Bt, np.kron(As, Br)) + np.kron(At, np.kron(Bs, Br)))


def _ext_1d(st_N, m, L, nbr, nface, e):
    out = []
    for axis in range(3):
        fl, fr = 2 * axis, 2 * axis + 1
        kl = schwarz.face_kind(st_N, m.dirichlet, nbr, e, fl)
        kr = schwarz.face_kind(st_N, m.dirichlet, nbr, e, fr)
        ll = L[nbr[e, fl], schwarz.FACES[nface[e, fl]][0]] if kl == "nbr" else L[e, axis]
        lr = L[nbr[e, fr], schwarz.FACES[nface[e, fr]][0]] if kr == "nbr" else L[e, axis]
        out.append(schwarz.extended_1d(st_N, ll, L[e, axis], lr, kl, kr))
    return out


def test_extension_is_lattice_neighbourhood():
    N = 3
    m = wl.box_mesh(3, 3, 3, N=N, hi=(1.0, 2.0, 0.5))
    nbr, nface = schwarz.face_neighbours(N, m.gid)
    ext = schwarz.extension_gids(N, m.gid, nbr, nface)
    gx = gy = 3 * N + 1
    e = 13  # centre element (1, 1, 1)
    NE = N + 3
    for c in range(NE):
        for b in range(NE):
            for a in range(NE):
                edge = sum(t in (0, NE - 1) for t in (a, b, c)) >= 2
                I, J, K = N - 1 + a, N - 1 + b, N - 1 + c
                want = -1 if edge else I + gx * (J + gy * K)
                assert ext[e, c, b, a] == want
    # a corner element has no layer across its boundary faces
    assert np.all(ext[0, :, :, 0] == -1) and np.all(ext[0, 0] == -1)


def _graded(m):
    """Piecewise-affine grading per direction: every element stays an affine brick,
    but neighbours along a line have different lengths."""
    m.x = np.interp(m.x, [0, 1 / 3, 2 / 3, 1], [0, 0.2, 0.7, 1.0])
    m.y = np.interp(m.y, [0, 1 / 3, 2 / 3, 1], [0, 0.9, 1.2, 2.0])
    m.z = np.interp(m.z, [0, 1 / 3, 2 / 3, 1], [0, 0.1, 0.35, 0.5])
    return m


def test_separable_operator_equals_assembled_on_affine_patch():
    N = 3
    m = _graded(wl.box_mesh(3, 3, 3, N=N))
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    Asp, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    nbr, nface = schwarz.face_neighbours(N, m.gid)
    L = schwarz.element_lengths(N, m.x, m.y, m.z)
    np.testing.assert_allclose(L[13], [0.5, 0.3, 0.25], rtol=1e-13)
    one_d = _ext_1d(N, m, L, nbr, nface, 13)
    K = _kron_op([o[0] for o in one_d], [o[1] for o in one_d])
    gx = gy = 3 * N + 1
    NE = N + 3
    box = [(N - 1 + a) + gx * ((N - 1 + b) + gy * (N - 1 + c)) for c in range(NE) for b in range(NE) for a in range(NE)]
    pos = np.searchsorted(ids, box)
    Asub = Asp[pos][:, pos].toarray()
    assert np.max(np.abs(K - Asub)) <= 1e-12 * np.max(np.abs(Asub))


@pytest.mark.parametrize("e", [13, 0, 5])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_fdm_solve_equals_dense_solve(e, dirichlet):
    N = 4
    m = wl.box_mesh(3, 3, 3, N=N, deform=0.05, seed=3, dirichlet=dirichlet)
    st = schwarz.setup(N, m.x, m.y, m.z, m.gid, m.dirichlet)
    nbr, nface = schwarz.face_neighbours(N, m.gid)
    L = schwarz.element_lengths(N, m.x, m.y, m.z)
    one_d = _ext_1d(N, m, L, nbr, nface, e)
    NE = N + 3
    act = np.zeros((NE, NE, NE), dtype=bool)
    lo = [o[2] for o in one_d]
    hi = [o[3] for o in one_d]
    act[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = True
    K = _kron_op([o[0] for o in one_d], [o[1] for o in one_d])
    a = act.ravel()
    rng = np.random.default_rng(e)
    b = np.where(act, rng.uniform(-1, 1, act.shape), 0.0)
    want = np.zeros(act.size)
    want[a] = np.linalg.solve(K[np.ix_(a, a)], b.ravel()[a])
    got = schwarz.fdm_solve(st.S[e], st.lam[e], b)
    assert np.max(np.abs(got.ravel() - want)) <= 1e-11 * np.max(np.abs(want))


def test_single_dirichlet_brick_is_solved_exactly():
    N = 5
    m = wl.box_mesh(1, N=N, hi=(1.0, 0.7, 1.3))
    G, B, _ = ops.geometric_factors(N, m.x, m.y, m.z)
    st = schwarz.setup(N, m.x, m.y, m.z, m.gid, m.dirichlet)
    r = wl.random_rhs(m, 1)
    z = schwarz.apply(st, r, "asm")
    Asp, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
    idsall, ru = ops.to_unique(m.gid, r)
    import scipy.sparse.linalg as spla
    x = ops.scatter_unique(m.gid, ids, spla.spsolve(Asp.tocsc(), ru[np.searchsorted(idsall, ids)]))
    assert np.max(np.abs(z - x)) <= 1e-11 * np.max(np.abs(x))
    assert np.max(np.abs(schwarz.apply(st, r, "ras") - x)) <= 1e-11 * np.max(np.abs(x))


def test_counting_function_matches_lattice_brute_force():
    N = 3
    nx, ny, nz = 3, 2, 2
    m = wl.box_mesh(nx, ny, nz, N=N)
    st = schwarz.setup(N, m.x, m.y, m.z, m.gid, m.dirichlet)
    gx, gy = nx * N + 1, ny * N + 1
    count = {}
    for ez in range(nz):
        for ey in range(ny):
            for ex in range(nx):
                for K in range(ez * N - 1, ez * N + N + 2):
                    for J in range(ey * N - 1, ey * N + N + 2):
                        for I in range(ex * N - 1, ex * N + N + 2):
                            ov = [I in (ex * N - 1, ex * N + N + 1), J in (ey * N - 1, ey * N + N + 1),
                                  K in (ez * N - 1, ez * N + N + 1)]
                            if sum(ov) >= 2:
                                continue  # edge or corner of the extended box
                            if not (0 < I < nx * N and 0 < J < ny * N and 0 < K < nz * N):
                                continue  # outside the mesh or on the Dirichlet boundary
                            g = I + gx * (J + gy * K)
                            count[g] = count.get(g, 0) + 1
    for g, w in zip(st.ids, st.weight_asm):
        c = count.get(int(g), 0)
        assert (w == 0 and c == 0) or abs(w - 1.0 / c) <= 1e-15


def test_unweighted_additive_schwarz_is_symmetric():
    N = 3
    m = wl.box_mesh(3, 2, 2, N=N, deform=0.05, seed=8)
    st = schwarz.setup(N, m.x, m.y, m.z, m.gid, m.dirichlet)
    u, v = wl.random_rhs(m, 1), wl.random_rhs(m, 2)
    su, sv = schwarz.apply(st, u, "sum"), schwarz.apply(st, v, "sum")
    a, b = ops.dot(m.gid, su, v), ops.dot(m.gid, u, sv)
    assert abs(a - b) <= 1e-12 * abs(a)
    assert ops.dot(m.gid, su, u) > 0


@pytest.mark.parametrize("variant", ["asm", "ras"])
def test_schwarz_smoothed_pmg_converges_faster_than_jacobi(variant):
    """The Schwarz-smoothed V-cycle as a FlexCG preconditioner reaches the
    direct solution in fewer iterations than the Chebyshev-Jacobi one."""
    from oracle import pmg, solvers as sv
    import scipy.sparse.linalg as spla
    N = 5
    m = wl.box_mesh(3, 3, 2, N=N, deform=0.05, seed=9)
    b = wl.random_rhs(m, 3)
    its = {}
    for sm in ("jacobi", variant):
        lv = pmg.build_levels(N, m.x, m.y, m.z, m.gid, m.dirichlet, smoother=sm)
        o = pmg.VCycleOpts(coarse_exact=True)
        res = pmg.pmg_flexcg(lv, b, o, rtol=1e-10)
        its[sm] = res.iters
        G = lv[0].G
        Asp, ids, _ = ops.assemble(N, G, m.gid, m.dirichlet)
        idsall, bu = ops.to_unique(m.gid, b)
        x = ops.scatter_unique(m.gid, ids, spla.spsolve(Asp.tocsc(), bu[np.searchsorted(idsall, ids)]))
        assert np.max(np.abs(res.x - x)) <= 1e-8 * np.max(np.abs(x))
    assert its[variant] < its["jacobi"]


def test_schwarz_invariant_under_element_rotations():
    """Turning elements' local numbering (every relative face orientation)
    leaves the operator unchanged, compared by global ID."""
    N = 3
    m = wl.box_mesh(3, 2, 2, N=N, deform=0.05, seed=2)
    r = wl.rotate_elements(m, 5)
    vals = np.random.default_rng(0).uniform(-1, 1, size=int(m.gid.max()) + 1)
    out = []
    for mm in (m, r):
        st = schwarz.setup(N, mm.x, mm.y, mm.z, mm.gid, mm.dirichlet)
        u = vals[mm.gid] * (mm.dirichlet == 0)
        for variant in ("asm", "ras"):
            z = schwarz.apply(st, u, variant)
            out.append(dict(zip(mm.gid.ravel().tolist(), z.ravel().tolist())))
    for a, b in ((out[0], out[2]), (out[1], out[3])):
        assert max(abs(a[g] - b[g]) for g in a) <= 1e-13

"""p-multigrid hierarchy and V-cycle (oracle, FP64).

Test infrastructure: see the package docstring.

The paper's pMG (Implementation, pMG paragraph): coarse-to-fine interpolation
is the tensor contraction u_f = (Jhat x Jhat x Jhat) u_c with one 1D Jhat per
level pair; smoothing by Chebyshev-accelerated point Jacobi; all pMG steps in
32-bit (this oracle stays in FP64; the FP32 GPU path is compared against it
with a tolerance). The smoother is Chebyshev-accelerated point Jacobi or
Chebyshev-accelerated overlapping Schwarz (oracle.schwarz). The coarsest level (N=1) is solved by Jacobi-PCG to a loose
relative tolerance, standing in for the paper's CPU AMG coarse solve.

Readings taken where the paper is silent:
  * coarse operators are re-discretised SEM Laplacians at the coarse order on
    the fine isoparametric map evaluated at the coarse GLL points;
  * restriction is the transpose of prolongation in the unique-DOF inner
    product: r_c = M_c QQ^T_c (Jhat^T x Jhat^T x Jhat^T)(r_f / mult_f);
  * a smoothing sweep is one Chebyshev cycle of degree k on [lo rho, hi rho];
    pre-smoothing starts from 0, post-smoothing from the corrected iterate.

Coarse connectivity is found here by matching coarse node coordinates (an
independent route from the HIP library, which keys coarse nodes by mesh
entities of the fine global IDs).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from . import operators as ops
from . import schwarz
from . import solvers
from .counter_rng import start_vector
from .reference_ops import gll, interp_matrix, prolongation_1d


@dataclass
class Level:
    N: int
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    gid: np.ndarray
    dirichlet: np.ndarray
    G: np.ndarray = None
    B: np.ndarray = None
    dinv: np.ndarray = None
    mult: np.ndarray = None
    rho: float = None
    extra: dict = field(default_factory=dict)

    def A(self, u):
        return ops.apply_A(self.N, self.G, self.gid, self.dirichlet, u)

    def dot(self, a, b):
        return float(np.sum(a * b / self.mult))

    def M(self, v):
        """The smoother's preconditioner: D^-1 (Jacobi) or the Schwarz operator."""
        st = self.extra.get("schwarz")
        if st is None:
            return self.dinv * v
        return schwarz.apply(st, v, self.extra["schwarz_variant"])


def tensor_apply(M: np.ndarray, u: np.ndarray, n_in: int) -> np.ndarray:
    """(M x M x M) u per element; u is [E, n_in^3], M is [n_out, n_in]."""
    E = u.shape[0]
    n_out = M.shape[0]
    u4 = u.reshape(E, n_in, n_in, n_in)
    a = np.matmul(u4, M.T)                                  # along i
    a = np.matmul(M, a)                                     # along j  -> [E, n_in, n_out, n_out]
    a = np.matmul(M, a.reshape(E, n_in, n_out * n_out))     # along k
    return a.reshape(E, n_out ** 3)


def coarse_coordinates(Nf, Nc, x, y, z):
    """Fine isoparametric map evaluated at the coarse GLL points."""
    Jcf = interp_matrix(gll(Nf)[0], gll(Nc)[0])  # (Nc+1) x (Nf+1)
    return tuple(tensor_apply(Jcf, c, Nf + 1) for c in (x, y, z))


def match_ids(x, y, z, tol):
    """Global IDs by clustering coincident nodes (distance <= tol)."""
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    tree = cKDTree(pts)
    pairs = tree.query_pairs(r=tol, output_type="ndarray")
    n = pts.shape[0]
    g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
    _, labels = connected_components(g, directed=False)
    return labels.astype(np.int64).reshape(x.shape)


def coarse_dirichlet(Nf, Nc, dir_f):
    """A coarse node is Dirichlet iff every fine node of the same element entity
    (vertex, edge, face or interior, in that element) is Dirichlet."""
    nf, nc = Nf + 1, Nc + 1
    E = dir_f.shape[0]
    df = dir_f.reshape(E, nf, nf, nf).astype(bool)  # [e, k, j, i]
    out = np.zeros((E, nc, nc, nc), dtype=np.uint8)

    def fine_range(ic):
        if ic == 0:
            return [0]
        if ic == Nc:
            return [Nf]
        return list(range(1, Nf))

    for kc in range(nc):
        for jc in range(nc):
            for ic in range(nc):
                ks, js, is_ = fine_range(kc), fine_range(jc), fine_range(ic)
                sub = df[:, ks][:, :, js][:, :, :, is_]
                out[:, kc, jc, ic] = np.all(sub.reshape(E, -1), axis=1)
    return out.reshape(E, nc ** 3)


def build_levels(N, x, y, z, gid, dirichlet, orders=None, rho=None, power_iters=20, smoother="jacobi"):
    """Levels finest-first. rho: optional list of overrides (one per smoothed level).

    smoother: "jacobi" (Chebyshev-Jacobi), "asm" or "ras" (Chebyshev-accelerated
    overlapping Schwarz with FDM local solves, see oracle.schwarz); rho is then
    the largest eigenvalue estimate of M A for that M.
    """
    if orders is None:
        orders = [N, (N - 1) // 2, 1] if N > 2 else [N, 1]
    assert orders[0] == N and orders[-1] == 1
    scale = max(np.ptp(x), np.ptp(y), np.ptp(z))
    levels = []
    for li, Nl in enumerate(orders):
        if li == 0:
            lev = Level(Nl, x, y, z, gid, dirichlet)
        else:
            prev = levels[-1]
            xc, yc, zc = coarse_coordinates(prev.N, Nl, prev.x, prev.y, prev.z)
            gc = match_ids(xc, yc, zc, 1e-9 * scale)
            dc = coarse_dirichlet(prev.N, Nl, prev.dirichlet)
            lev = Level(Nl, xc, yc, zc, gc, dc)
            lev_J = prolongation_1d(Nl, prev.N)
            prev.extra["J_from_coarse"] = lev_J
        lev.G, lev.B, _ = ops.geometric_factors(lev.N, lev.x, lev.y, lev.z)
        lev.mult = ops.multiplicity(lev.gid)
        lev.dinv = ops.jacobi_inverse(lev.N, lev.G, lev.gid, lev.dirichlet)
        levels.append(lev)
    for li, lev in enumerate(levels[:-1]):
        if smoother != "jacobi":
            lev.extra["schwarz"] = schwarz.setup(lev.N, lev.x, lev.y, lev.z, lev.gid, lev.dirichlet)
            lev.extra["schwarz_variant"] = smoother
        if rho is not None and rho[li] is not None:
            lev.rho = float(rho[li])
        else:
            v0 = ops.mask(lev.dirichlet, start_vector(lev.gid))
            if smoother == "jacobi":
                lev.rho = solvers.power_rho(lev.A, lev.dinv, lev.dot, v0, iters=power_iters)
            else:
                lev.rho = schwarz.power_rho(lev.A, lev.M, lev.dot, v0, iters=power_iters)
    return levels


def prolong(levels, l, zc):
    """Coarse level l+1 -> fine level l: (Jhat x Jhat x Jhat) per element."""
    J = levels[l].extra["J_from_coarse"]
    return tensor_apply(J, zc, levels[l + 1].N + 1)


def restrict(levels, l, rf):
    """Fine level l -> coarse level l+1: M_c QQ^T_c (Jhat^T)^{x3} (r_f / mult_f)."""
    J = levels[l].extra["J_from_coarse"]
    c = levels[l + 1]
    rc = tensor_apply(J.T, rf / levels[l].mult, levels[l].N + 1)
    return ops.mask(c.dirichlet, ops.gs(c.gid, rc))


@dataclass
class VCycleOpts:
    degree: int = 2
    pre: int = 1
    post: int = 1
    lo: float = 0.1
    hi: float = 1.1
    coarse_rtol: float = 1e-2
    coarse_maxit: int = 500
    coarse_fixed_iters: int | None = None
    coarse_exact: bool = False


def coarse_solve(lev: Level, r, o: VCycleOpts):
    if o.coarse_exact:
        A, ids, _ = ops.assemble(lev.N, lev.G, lev.gid, lev.dirichlet)
        from scipy.sparse.linalg import spsolve
        _, rv = ops.to_unique(lev.gid, r)
        idsall, _ = ops.unique_index(lev.gid)
        rin = rv[np.searchsorted(idsall, ids)]
        xin = spsolve(A.tocsc(), rin)
        return ops.scatter_unique(lev.gid, ids, xin)
    res = solvers.pcg(lev.A, lambda v: lev.dinv * v, lev.dot, r, rtol=o.coarse_rtol,
                      maxit=o.coarse_maxit, fixed_iters=o.coarse_fixed_iters)
    return res.x


def vcycle(levels, r, o: VCycleOpts, l: int = 0):
    lev = levels[l]
    if l == len(levels) - 1:
        return coarse_solve(lev, r, o)
    z = None
    for _ in range(o.pre):
        z = solvers.chebyshev(lev.A, lev.M, r, lev.rho, o.degree, o.lo, o.hi, x0=z)
    e = r - lev.A(z) if z is not None else r.copy()
    zc = vcycle(levels, restrict(levels, l, e), o, l + 1)
    zp = prolong(levels, l, zc)
    z = zp if z is None else z + zp
    for _ in range(o.post):
        z = solvers.chebyshev(lev.A, lev.M, r, lev.rho, o.degree, o.lo, o.hi, x0=z)
    return z


def pmg_flexcg(levels, b, o: VCycleOpts = None, rtol=1e-8, maxit=200, fixed_iters=None):
    o = o or VCycleOpts()
    top = levels[0]
    return solvers.flexcg(top.A, lambda r: vcycle(levels, r, o), top.dot, b, rtol=rtol,
                          maxit=maxit, fixed_iters=fixed_iters)

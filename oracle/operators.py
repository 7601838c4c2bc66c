"""SEM operators on element-local storage (oracle, FP64).

Test infrastructure: see the package docstring.

Storage: a field is an "E-vector" u[e, p], p = i + (N+1) j + (N+1)^2 k, i.e. the
(N+1)^3 GLL values of each element with i (the r direction) fastest
(Algorithms: local i-j-k indexing). Internally arrays are viewed as
u[e, k, j, i].

Definitions (the paper names the Poisson operator "Ax" and writes only the
basis and the derivative footnote, Algorithms, eq. field1; the textbook weak
form with GLL quadrature collocated at the nodes is used):
  * isoparametric map x^e(r,s,t) = sum_ijk x^e_ijk h_i(r) h_j(s) h_k(t);
    Jacobian matrix Jm[l][m] = d x_l / d r_m obtained by applying Dhat along
    each direction to the nodal coordinates;
  * G_mn = W |J| sum_l (d r_m / d x_l)(d r_n / d x_l), m, n in {r, s, t},
    stored as rr, rs, rt, ss, st, tt; B = W |J|; W = w_i w_j w_k;
  * local Ax: (A_L u) = sum_m D_m^T ( sum_n G_mn D_n u ), with D_r, D_s, D_t
    Dhat applied along i, j, k;
  * gather-scatter QQ^T: every copy of a global node receives the sum over all
    copies (Implementation, Autotuned Communication: exchange-and-sum of
    shared interface values keyed by a global ID per vertex);
  * mask M: zero the copies of Dirichlet nodes;
  * assembled operator A = M QQ^T A_L on consistent masked E-vectors;
  * inner product over unique DOFs: (x, y) = sum_l x_l y_l / mult_l.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .reference_ops import gll, deriv_matrix

G_NAMES = ("rr", "rs", "rt", "ss", "st", "tt")
# (m, n) -> slot in the 6-component symmetric storage
_SLOT = {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}


def slot(m: int, n: int) -> int:
    return _SLOT[(min(m, n), max(m, n))]


def _as4(u: np.ndarray, N: int) -> np.ndarray:
    n = N + 1
    return u.reshape(-1, n, n, n)


def grad_ref(N: int, u: np.ndarray, D: np.ndarray | None = None):
    """(u_r, u_s, u_t) on every element: Dhat applied along i, j and k."""
    if D is None:
        D = deriv_matrix(N)
    n = N + 1
    u4 = _as4(u, N)
    ur = np.matmul(u4, D.T)                      # sum_a D[i,a] u[e,k,j,a]
    us = np.matmul(D, u4)                        # sum_b D[j,b] u[e,k,b,i]
    ut = np.matmul(D, u4.reshape(-1, n, n * n)).reshape(u4.shape)  # sum_c D[k,c] u[e,c,j,i]
    return ur, us, ut


def grad_ref_transpose(N: int, wr, ws, wt, D: np.ndarray | None = None):
    """D_r^T wr + D_s^T ws + D_t^T wt on every element."""
    if D is None:
        D = deriv_matrix(N)
    n = N + 1
    out = np.matmul(wr, D)                       # sum_a D[a,i] wr[e,k,j,a]
    out = out + np.matmul(D.T, ws)               # sum_b D[b,j] ws[e,k,b,i]
    out = out + np.matmul(D.T, wt.reshape(-1, n, n * n)).reshape(wt.shape)
    return out


def geometric_factors(N: int, x: np.ndarray, y: np.ndarray, z: np.ndarray):
    """G [E, 6, Np], B [E, Np] and det J [E, Np] from nodal coordinates [E, Np]."""
    _, w = gll(N)
    n = N + 1
    E = x.shape[0]
    Jm = np.empty((E, n, n, n, 3, 3))
    for l, c in enumerate((x, y, z)):
        cr, cs, ct = grad_ref(N, c)
        Jm[..., l, 0] = cr
        Jm[..., l, 1] = cs
        Jm[..., l, 2] = ct
    detJ = np.linalg.det(Jm)
    if np.any(detJ <= 0):
        raise ValueError("non-positive Jacobian determinant")
    Jinv = np.linalg.inv(Jm)  # Jinv[..., m, l] = d r_m / d x_l
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :])  # [k, j, i]
    WJ = W[None] * detJ
    G = np.empty((E, 6, n, n, n))
    for m in range(3):
        for nn in range(m, 3):
            G[:, slot(m, nn)] = WJ * np.sum(Jinv[..., m, :] * Jinv[..., nn, :], axis=-1)
    return G.reshape(E, 6, n ** 3), WJ.reshape(E, n ** 3), detJ.reshape(E, n ** 3)


def ax_local(N: int, G: np.ndarray, u: np.ndarray) -> np.ndarray:
    """A_L u = sum_m D_m^T sum_n G_mn D_n u, element by element (no gs, no mask)."""
    n = N + 1
    E = u.shape[0]
    g = G.reshape(E, 6, n, n, n)
    grads = grad_ref(N, u)
    w = []
    for m in range(3):
        acc = np.zeros_like(grads[0])
        for nn in range(3):
            acc = acc + g[:, slot(m, nn)] * grads[nn]
        w.append(acc)
    return grad_ref_transpose(N, *w).reshape(E, n ** 3)


def helmholtz_local(N: int, G, B, lam: float, u):
    """(A_L + lam B) u, the velocity-substep Helmholtz operator."""
    return ax_local(N, G, u) + lam * B * u


# ---------------------------------------------------------------------------
# gather-scatter, mask, weights
# ---------------------------------------------------------------------------

def unique_index(gid: np.ndarray):
    """(ids, inverse) so that gid.ravel() == ids[inverse]."""
    ids, inv = np.unique(gid.ravel(), return_inverse=True)
    return ids, inv


def gs(gid: np.ndarray, v: np.ndarray) -> np.ndarray:
    """QQ^T v: each local copy receives the sum over all copies of its node."""
    _, inv = unique_index(gid)
    sums = np.bincount(inv, weights=v.ravel())
    return sums[inv].reshape(v.shape)


def multiplicity(gid: np.ndarray) -> np.ndarray:
    _, inv = unique_index(gid)
    cnt = np.bincount(inv)
    return cnt[inv].reshape(gid.shape).astype(np.float64)


def mask(dirichlet: np.ndarray, v: np.ndarray) -> np.ndarray:
    return np.where(dirichlet != 0, 0.0, v)


def dot(gid: np.ndarray, a: np.ndarray, b: np.ndarray) -> float:
    """Inner product over unique DOFs of two consistent E-vectors."""
    return float(np.sum(a * b / multiplicity(gid)))


def to_unique(gid: np.ndarray, v: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(ids, values) of a consistent E-vector, one value per unique ID (first copy)."""
    ids, first = np.unique(gid.ravel(), return_index=True)
    return ids, v.ravel()[first]


def apply_A(N, G, gid, dirichlet, u):
    """Assembled, masked operator on a consistent E-vector: M QQ^T A_L u."""
    return mask(dirichlet, gs(gid, ax_local(N, G, u)))


# ---------------------------------------------------------------------------
# Jacobi diagonal
# ---------------------------------------------------------------------------

def diag_local(N: int, G: np.ndarray) -> np.ndarray:
    """Diagonal of each element matrix A^e = sum_mn D_m^T diag(G_mn) D_n.

    At point (i,j,k):
      sum_a D[a,i]^2 G_rr(a,j,k) + sum_b D[b,j]^2 G_ss(i,b,k) + sum_c D[c,k]^2 G_tt(i,j,c)
      + 2 D[i,i] D[j,j] G_rs + 2 D[i,i] D[k,k] G_rt + 2 D[j,j] D[k,k] G_st  (at (i,j,k)).
    """
    D = deriv_matrix(N)
    n = N + 1
    E = G.shape[0]
    g = G.reshape(E, 6, n, n, n)
    D2 = D * D
    d = np.matmul(g[:, 0], D2)                                   # sum_a D[a,i]^2 Grr[e,k,j,a]
    d = d + np.matmul(D2.T, g[:, 3])                             # sum_b D[b,j]^2 Gss[e,k,b,i]
    d = d + np.matmul(D2.T, g[:, 5].reshape(E, n, n * n)).reshape(E, n, n, n)
    dd = np.diag(D)
    di = dd[None, None, None, :]
    dj = dd[None, None, :, None]
    dk = dd[None, :, None, None]
    d = d + 2 * di * dj * g[:, 1] + 2 * di * dk * g[:, 2] + 2 * dj * dk * g[:, 4]
    return d.reshape(E, n ** 3)


def jacobi_inverse(N, G, gid, dirichlet) -> np.ndarray:
    """1 / diag(A) on consistent storage, 0 on Dirichlet nodes."""
    d = gs(gid, diag_local(N, G))
    inv = np.where(dirichlet != 0, 0.0, 1.0 / np.where(dirichlet != 0, 1.0, d))
    return inv


# ---------------------------------------------------------------------------
# Assembled sparse matrix (tiny meshes only)
# ---------------------------------------------------------------------------

def element_matrices(N: int, G: np.ndarray) -> np.ndarray:
    """Dense A^e = sum_mn Dm^T diag(G_mn) Dn with Kronecker-product Dm ([E, Np, Np])."""
    D = deriv_matrix(N)
    I = np.eye(N + 1)
    Dm = [np.kron(I, np.kron(I, D)), np.kron(I, np.kron(D, I)), np.kron(D, np.kron(I, I))]
    E, _, Np = G.shape
    A = np.zeros((E, Np, Np))
    for m in range(3):
        for n in range(3):
            A += np.matmul(Dm[m].T[None] * G[:, slot(m, n)][:, None, :], Dm[n])
    return A


def assemble(N: int, G: np.ndarray, gid: np.ndarray, dirichlet: np.ndarray,
             B: np.ndarray | None = None):
    """Assembled stiffness Q^T blockdiag(A^e) Q on interior unique DOFs.

    Returns (A_csr, ids_interior, B_diag_interior or None). Row/column r
    corresponds to global ID ids_interior[r].
    """
    Ae = element_matrices(N, G)
    ids, inv = unique_index(gid)
    inv = inv.reshape(gid.shape)
    E, Np = gid.shape
    rows = np.repeat(inv[:, :, None], Np, axis=2).ravel()
    cols = np.repeat(inv[:, None, :], Np, axis=1).ravel()
    n = len(ids)
    A = sp.coo_matrix((Ae.ravel(), (rows, cols)), shape=(n, n)).tocsr()
    dflag = np.zeros(n, dtype=bool)
    dflag[inv.ravel()[dirichlet.ravel() != 0]] = True
    keep = np.nonzero(~dflag)[0]
    A = A[keep][:, keep]
    Bd = None
    if B is not None:
        Bd = np.bincount(inv.ravel(), weights=B.ravel(), minlength=n)[keep]
    return A.tocsr(), ids[keep], Bd


def scatter_unique(gid: np.ndarray, ids: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """E-vector holding vals[r] at every copy of ids[r] (0 for IDs not listed)."""
    pos = np.searchsorted(ids, gid.ravel())
    pos = np.clip(pos, 0, len(ids) - 1)
    hit = ids[pos] == gid.ravel()
    out = np.where(hit, vals[pos], 0.0)
    return out.reshape(gid.shape)


def assemble_rhs(N, B, gid, dirichlet, f):
    """b = M QQ^T (B f): weak form of a nodal source f."""
    return mask(dirichlet, gs(gid, B * f))


# ---------------------------------------------------------------------------
# Helmholtz (velocity substep operator, Implementation, Helmholtz paragraph)
# ---------------------------------------------------------------------------

def apply_H(N, G, B, lam, gid, dirichlet, u):
    """M QQ^T (A_L + lam B) u on a consistent E-vector."""
    return mask(dirichlet, gs(gid, helmholtz_local(N, G, B, lam, u)))


def helmholtz_jacobi_inverse(N, G, B, lam, gid, dirichlet) -> np.ndarray:
    """1 / diag(A + lam B) on consistent storage, 0 on Dirichlet nodes."""
    d = gs(gid, diag_local(N, G) + lam * B)
    return np.where(dirichlet != 0, 0.0, 1.0 / np.where(dirichlet != 0, 1.0, d))


def assemble_helmholtz(N, G, B, lam, gid, dirichlet):
    """Assembled A + lam diag(QQ^T B) on interior unique DOFs (tiny meshes)."""
    A, ids, Bd = assemble(N, G, gid, dirichlet, B)
    return (A + lam * sp.diags(Bd)).tocsr(), ids

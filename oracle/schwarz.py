"""Overlapping Schwarz smoother with fast-diagonalization local solves (oracle, FP64).

Test infrastructure: see the package docstring.

Implementation section, pMG smoothers and eq. fdm: each element is extended by
one node layer into its face neighbours, so an (N+1)^3 element gives an
(N+3)^3 local box; the local Poisson problem on it is solved by fast
diagonalization, u = (S_t x S_s x S_r) Lambda^-1 (S_t^T x S_s^T x S_r^T) b,
with one small matrix of 1D eigenvectors per direction and the eigenvalue sums
on the diagonal of Lambda. Only face data are exchanged to build the
extension (the 12 edge lines and 8 corners of the box are not filled). The
restricted variant (RAS) keeps only each element's own nodes of its local
solution.

Readings taken where the paper is silent (the construction follows the
hybrid Schwarz/multigrid smoothers of Lottes and Fischer, 2005):
  * faces are numbered -r, +r, -s, +s, -t, +t; the face-local coordinates
    (u, v) are (j, k) on r faces, (i, k) on s faces and (i, j) on t faces;
    two elements are face neighbours when they share the four corner global
    IDs of a face;
  * extension: the layer across face f of element e holds, for each node of
    that face, the neighbour's node one step into the neighbour behind the
    neighbour's copy of that face node (matched by global ID);
  * local operator: the separable Laplacian
        A~ = B_t (x) B_s (x) A_r + B_t (x) A_s (x) B_r + A_t (x) B_s (x) B_r
    built from 1D GLL stiffness A = (2/l) Dhat^T W Dhat and mass B = (l/2) W;
    l is the element's mean length in that direction (mean distance between
    the end nodes of its (N+1)^2 grid lines); along each direction the 1D
    operator is assembled over the element (ext nodes 1..N+1) and, across a
    face with a neighbour, the neighbour's last interval pair (ext nodes 0, 1
    on the left, N+1, N+2 on the right, neighbour length along that line),
    with homogeneous Dirichlet conditions beyond the extension;
  * boundary faces without a neighbour: if every node of the face is
    Dirichlet, the face node is excluded as well (active 1D range starts at
    ext node 2, or ends at N); otherwise the face node is kept with a natural
    (Neumann) end (range starts at 1, or ends at N+1);
  * additive Schwarz (ASM): z = W (.) sum_e R_e^T A~_e^-1 R_e r, where R_e
    gathers the subdomain values by global ID and R_e^T adds the local
    solution back at the same global IDs; W = 1 / c with the counting
    function c = sum_e R_e^T R_e 1 restricted to active positions;
  * RAS: z = (1 / mult) (.) sum_e R_e,own^T A~_e^-1 R_e r, keeping only each
    element's own (N+1)^3 nodes;
  * the result is masked (Dirichlet copies zero);
  * Chebyshev acceleration (the paper's Chebyshev-accelerated Schwarz) is the
    Chebyshev recurrence of solvers.chebyshev with D^-1 replaced by this
    operator; its rho is the power-iteration estimate |M A v| with |v| = 1
    after the given number of normalised iterations v <- M A v / |M A v|.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import operators as ops
from .reference_ops import deriv_matrix, gll

# face f -> (axis, side): axis 0 = r (i), 1 = s (j), 2 = t (k); side 0 = low, 1 = high
FACES = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]


def face_node(N, f, u, v, depth=0):
    """(i, j, k) of face-local node (u, v) of face f at the given depth into the element."""
    axis, side = FACES[f]
    d = depth if side == 0 else N - depth
    if axis == 0:
        return d, u, v
    if axis == 1:
        return u, d, v
    return u, v, d


def _p(N, i, j, k):
    n = N + 1
    return i + n * j + n * n * k


def face_neighbours(N, gid):
    """nbr[e, f] (element across face f, -1 if none) and nface[e, f] (its face)."""
    E = gid.shape[0]
    corners = {}
    key_of = {}
    for e in range(E):
        for f in range(6):
            key = tuple(sorted(int(gid[e, _p(N, *face_node(N, f, u, v))]) for u in (0, N) for v in (0, N)))
            key_of[(e, f)] = key
            corners.setdefault(key, []).append((e, f))
    nbr = -np.ones((E, 6), dtype=np.int64)
    nface = -np.ones((E, 6), dtype=np.int64)
    for (e, f), key in key_of.items():
        others = [(e2, f2) for (e2, f2) in corners[key] if (e2, f2) != (e, f)]
        if others:
            nbr[e, f], nface[e, f] = others[0]
    return nbr, nface


def extension_gids(N, gid, nbr, nface):
    """ext[e, c, b, a] = global ID at ext position (a, b, c), -1 outside the subdomain.

    Own nodes sit at (i+1, j+1, k+1); face layers at a = 0 / N+2 (r faces), etc.
    """
    E = gid.shape[0]
    NE = N + 3
    ext = -np.ones((E, NE, NE, NE), dtype=np.int64)
    g4 = gid.reshape(E, N + 1, N + 1, N + 1)  # [e, k, j, i]
    ext[:, 1:N + 2, 1:N + 2, 1:N + 2] = g4
    for e in range(E):
        for f in range(6):
            n, fn = nbr[e, f], nface[e, f]
            if n < 0:
                continue
            # where each global ID of the neighbour's face fn sits (face coords)
            pos = {}
            for u in range(N + 1):
                for v in range(N + 1):
                    pos[int(gid[n, _p(N, *face_node(N, fn, u, v))])] = (u, v)
            axis, side = FACES[f]
            layer = 0 if side == 0 else N + 2
            for u in range(N + 1):
                for v in range(N + 1):
                    g = int(gid[e, _p(N, *face_node(N, f, u, v))])
                    un, vn = pos[g]
                    gn = int(gid[n, _p(N, *face_node(N, fn, un, vn, depth=1))])
                    if axis == 0:
                        ext[e, v + 1, u + 1, layer] = gn
                    elif axis == 1:
                        ext[e, v + 1, layer, u + 1] = gn
                    else:
                        ext[e, layer, v + 1, u + 1] = gn
    return ext


def element_lengths(N, x, y, z):
    """[E, 3]: mean distance between the end nodes of the grid lines along r, s, t."""
    E = x.shape[0]
    n = N + 1
    X = np.stack([x, y, z], axis=-1).reshape(E, n, n, n, 3)  # [e, k, j, i, xyz]
    lr = np.linalg.norm(X[:, :, :, -1] - X[:, :, :, 0], axis=-1).mean(axis=(1, 2))
    ls = np.linalg.norm(X[:, :, -1, :] - X[:, :, 0, :], axis=-1).mean(axis=(1, 2))
    lt = np.linalg.norm(X[:, -1, :, :] - X[:, 0, :, :], axis=-1).mean(axis=(1, 2))
    return np.stack([lr, ls, lt], axis=1)


def face_kind(N, dirichlet, nbr, e, f):
    """'nbr', 'dir' (every face node Dirichlet) or 'neu'."""
    if nbr[e, f] >= 0:
        return "nbr"
    flags = [dirichlet[e, _p(N, *face_node(N, f, u, v))] for u in range(N + 1) for v in range(N + 1)]
    return "dir" if all(flags) else "neu"


def extended_1d(N, l_left, l_mid, l_right, kind_left, kind_right):
    """(A, B, lo, hi): 1D extended stiffness and mass on ext nodes 0..N+2 and the active range."""
    xi, w = gll(N)
    D = deriv_matrix(N)
    Ahat = D.T @ np.diag(w) @ D
    NE = N + 3
    A = np.zeros((NE, NE))
    B = np.zeros((NE, NE))
    A[1:N + 2, 1:N + 2] += (2.0 / l_mid) * Ahat
    B[1:N + 2, 1:N + 2] += (l_mid / 2.0) * np.diag(w)
    if kind_left == "nbr":
        A[0:2, 0:2] += (2.0 / l_left) * Ahat[N - 1:N + 1, N - 1:N + 1]
        B[0:2, 0:2] += (l_left / 2.0) * np.diag(w[N - 1:N + 1])
    if kind_right == "nbr":
        A[N + 1:N + 3, N + 1:N + 3] += (2.0 / l_right) * Ahat[0:2, 0:2]
        B[N + 1:N + 3, N + 1:N + 3] += (l_right / 2.0) * np.diag(w[0:2])
    lo = {"nbr": 0, "neu": 1, "dir": 2}[kind_left]
    hi = {"nbr": N + 2, "neu": N + 1, "dir": N}[kind_right]
    return A, B, lo, hi


def fdm_1d(A, B, lo, hi):
    """S (columns: B-orthonormal eigenvectors on the active range, zero elsewhere) and lam."""
    NE = A.shape[0]
    S = np.zeros((NE, NE))
    lam = np.ones(NE)
    act = slice(lo, hi + 1)
    if hi >= lo:
        vals, vecs = sla.eigh(A[act, act], B[act, act])  # library generalized eigensolver
        S[act, act] = vecs
        lam[act] = vals
    return S, lam


@dataclass
class SchwarzSetup:
    N: int
    gid: np.ndarray
    dirichlet: np.ndarray
    ext: np.ndarray        # [E, NE, NE, NE] global IDs, -1 outside
    active: np.ndarray     # [E, NE, NE, NE] bool: in the subdomain and in every active range
    S: list                # per element: (S_r, S_s, S_t)
    lam: list              # per element: (lam_r, lam_s, lam_t)
    ids: np.ndarray        # unique global IDs
    weight_asm: np.ndarray  # per unique ID: 1 / count (0 where count = 0)
    mult: np.ndarray       # per unique ID


def setup(N, x, y, z, gid, dirichlet):
    E = gid.shape[0]
    NE = N + 3
    nbr, nface = face_neighbours(N, gid)
    ext = extension_gids(N, gid, nbr, nface)
    L = element_lengths(N, x, y, z)
    S, lam = [], []
    active = np.zeros(ext.shape, dtype=bool)
    for e in range(E):
        Se, le, rng = [], [], []
        for axis in range(3):
            fl, fr = 2 * axis, 2 * axis + 1
            kl, kr = face_kind(N, dirichlet, nbr, e, fl), face_kind(N, dirichlet, nbr, e, fr)
            l_left = L[nbr[e, fl], FACES[nface[e, fl]][0]] if kl == "nbr" else L[e, axis]
            l_right = L[nbr[e, fr], FACES[nface[e, fr]][0]] if kr == "nbr" else L[e, axis]
            A1, B1, lo, hi = extended_1d(N, l_left, L[e, axis], l_right, kl, kr)
            s, lv = fdm_1d(A1, B1, lo, hi)
            Se.append(s)
            le.append(lv)
            rng.append(np.arange(NE)[(np.arange(NE) >= lo) & (np.arange(NE) <= hi)])
        S.append(tuple(Se))
        lam.append(tuple(le))
        m = np.zeros((NE, NE, NE), dtype=bool)  # [c, b, a]
        m[np.ix_(rng[2], rng[1], rng[0])] = True
        active[e] = m & (ext[e] >= 0)
    ids, inv = np.unique(gid, return_inverse=True)
    mult = np.bincount(inv.ravel(), minlength=len(ids)).astype(float)
    st = SchwarzSetup(N, gid, dirichlet, ext, active, S, lam, ids, None, mult)
    count = _accumulate(st, [np.where(st.active[e], 1.0, 0.0) for e in range(E)], own_only=False)
    st.weight_asm = np.where(count > 0, 1.0 / np.maximum(count, 1.0), 0.0)
    return st


def fdm_solve(S, lam, b):
    """(S_t x S_s x S_r) Lambda^-1 (S_t^T x S_s^T x S_r^T) b on an [c, b, a] box."""
    Sr, Ss, St = S
    lr, ls, lt = lam
    t = np.einsum("ca,zyc->zya", Sr, b)   # S_r^T along a
    t = np.einsum("cb,zca->zba", Ss, t)   # S_s^T along b
    t = np.einsum("cz,cba->zba", St, t)   # S_t^T along c
    Lam = lt[:, None, None] + ls[None, :, None] + lr[None, None, :]
    t = np.where(Lam > 0, t / np.where(Lam > 0, Lam, 1.0), 0.0)
    t = np.einsum("ac,zyc->zya", Sr, t)
    t = np.einsum("bc,zca->zba", Ss, t)
    t = np.einsum("zc,cba->zba", St, t)
    return t


def _accumulate(st, local, own_only):
    """sum_e R_e^T local_e over unique IDs (positions outside the subdomain dropped)."""
    N = st.N
    acc = np.zeros(len(st.ids))
    for e, u in enumerate(local):
        keep = st.ext[e] >= 0
        if own_only:
            own = np.zeros_like(keep)
            own[1:N + 2, 1:N + 2, 1:N + 2] = True
            keep &= own
        idx = np.searchsorted(st.ids, st.ext[e][keep])
        np.add.at(acc, idx, u[keep])
    return acc


def apply(st, r, variant="asm", local="fdm"):
    """z = Schwarz(r) on a consistent masked E-vector r (see the module docstring)."""
    N = st.N
    E = r.shape[0]
    ids, first = np.unique(st.gid.ravel(), return_index=True)
    runiq = r.ravel()[first]
    local_sol = []
    for e in range(E):
        b = np.zeros(st.ext[e].shape)
        inside = st.ext[e] >= 0
        b[inside] = runiq[np.searchsorted(ids, st.ext[e][inside])]
        b = np.where(st.active[e], b, 0.0)
        if local == "fdm":
            u = fdm_solve(st.S[e], st.lam[e], b)
        else:
            u = b
        local_sol.append(np.where(st.active[e], u, 0.0))
    if variant == "asm":
        zu = st.weight_asm * _accumulate(st, local_sol, own_only=False)
    elif variant == "ras":
        zu = _accumulate(st, local_sol, own_only=True) / st.mult
    elif variant == "sum":  # unweighted additive Schwarz (for the symmetry pin)
        zu = _accumulate(st, local_sol, own_only=False)
    else:
        raise ValueError(variant)
    z = ops.scatter_unique(st.gid, ids, zu)
    return ops.mask(st.dirichlet, z)


def power_rho(apply_A, apply_M, dot, v0, iters=20):
    """|M A v| after `iters` normalised power iterations from v0."""
    v = v0 / np.sqrt(dot(v0, v0))
    for _ in range(iters):
        w = apply_M(apply_A(v))
        v = w / np.sqrt(dot(w, w))
    w = apply_M(apply_A(v))
    return float(np.sqrt(dot(w, w)))

"""Seeded synthetic inputs for the SEM Poisson solve (meshes and right-hand sides).

This module holds the input generators shared by the tests, the benchmark and
the serving loop. It contains none of the method's arithmetic: it places mesh
nodes, labels them with global IDs and Dirichlet flags, and draws random
right-hand sides. Everything the method computes from these arrays (reference
operators, geometric factors, Ax, gather-scatter, solvers) lives elsewhere.

The paper's workloads are reactor meshes (pebble beds, rod bundles) of
curvilinear hex elements at N=7-8 (Introduction; Performance Results) that are
not available here. Deformed boxes of hex elements stand in for them:

* the unit cube is split into nx*ny*nz bricks;
* each brick carries an (N+1)^3 tensor grid of nodes placed at the
  Gauss-Lobatto points of each direction (computed here with numpy's Legendre
  root finder, endpoints set to exactly -1 and +1 so that nodes shared by two
  bricks are bitwise equal);
* optionally every node is moved by the smooth map
      x_i <- x_i + a * sin(2 pi x_j + phi_i1) * sin(2 pi x_k + phi_i2),
  (i, j, k) cyclic, with phases phi drawn from default_rng(seed);
* global IDs number the lattice points of the box; Dirichlet flags mark the
  outer faces.

Where the nodes are placed only fixes the shape of the domain: the method reads
the nodal coordinates as the definition of the isoparametric map of each
element (Algorithms, eq. field1), so a node placed slightly off a Gauss-Lobatto
point changes the geometry, not the correctness of any step.

Arrays use element-local ("E-vector") layout: shape [E, (N+1)^3] with the local
index p = i + (N+1) j + (N+1)^2 k, i (the r direction) fastest.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "BoxMesh",
    "box_mesh",
    "random_rhs",
    "manufactured_source",
    "manufactured_solution",
    "manufactured_neumann_solution",
    "relabel",
    "rotate_elements",
    "config_meshes",
    "batched_problem_specs",
    "serving_mesh_sides",
    "rhs_sequence",
    "rhs_sequence_fn",
]


@dataclass
class BoxMesh:
    """Host arrays describing one hex mesh (all C-contiguous)."""

    N: int
    shape: tuple  # (nx, ny, nz) elements per direction
    x: np.ndarray  # [E, (N+1)^3] float64
    y: np.ndarray
    z: np.ndarray
    gid: np.ndarray  # [E, (N+1)^3] int64, global node IDs (>= 0)
    dirichlet: np.ndarray  # [E, (N+1)^3] uint8, 1 on the outer boundary
    deform: float = 0.0
    seed: int | None = None
    meta: dict = field(default_factory=dict)

    @property
    def E(self) -> int:
        return self.x.shape[0]

    @property
    def Np(self) -> int:
        return (self.N + 1) ** 3

    @property
    def n_local(self) -> int:
        return self.E * self.Np


def _node_positions_1d(N: int) -> np.ndarray:
    """Positions of N+1 nodes on [-1, 1]: the endpoints and the roots of P_N'.

    Uses numpy's Legendre class (a library root finder). The endpoints are
    exact, the interior roots are symmetrised so the grid is mirror-symmetric.
    """
    if N == 1:
        return np.array([-1.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(N).deriv().roots().real
    inner = np.sort(inner)
    inner = 0.5 * (inner - inner[::-1])  # exact mirror symmetry
    pts = np.concatenate(([-1.0], inner, [1.0]))
    return pts


def box_mesh(nx: int, ny: int | None = None, nz: int | None = None, *, N: int = 7,
             deform: float = 0.0, seed: int = 0, dirichlet: bool = True,
             lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> BoxMesh:
    """Deformed-box mesh of nx*ny*nz hex elements of order N.

    Element e = ex + nx*(ey + ny*ez). deform is the amplitude a of the smooth
    map described in the module docstring (0 gives straight bricks).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    if N < 1:
        raise ValueError("N must be >= 1")
    NP = N + 1
    xi = _node_positions_1d(N)
    t = 0.5 * (xi + 1.0)  # in [0, 1], exact endpoints

    E = nx * ny * nz
    ex = np.arange(E) % nx
    ey = (np.arange(E) // nx) % ny
    ez = np.arange(E) // (nx * ny)

    # lattice coordinates (integers) of every local node
    li = np.arange(NP)
    I = (ex[:, None, None, None] * N + li[None, None, None, :])
    J = (ey[:, None, None, None] * N + li[None, None, :, None])
    K = (ez[:, None, None, None] * N + li[None, :, None, None])
    I = np.broadcast_to(I, (E, NP, NP, NP))
    J = np.broadcast_to(J, (E, NP, NP, NP))
    K = np.broadcast_to(K, (E, NP, NP, NP))

    # unit-cube positions: (e_d + t_i) / n_d, same expression on both sides of a face
    ux = (ex[:, None, None, None] + t[None, None, None, :]) / nx
    uy = (ey[:, None, None, None] + t[None, None, :, None]) / ny
    uz = (ez[:, None, None, None] + t[None, :, None, None]) / nz
    ux = np.broadcast_to(ux, (E, NP, NP, NP))
    uy = np.broadcast_to(uy, (E, NP, NP, NP))
    uz = np.broadcast_to(uz, (E, NP, NP, NP))

    X = lo[0] + (hi[0] - lo[0]) * ux
    Y = lo[1] + (hi[1] - lo[1]) * uy
    Z = lo[2] + (hi[2] - lo[2]) * uz

    if deform != 0.0:
        rng = np.random.default_rng(seed)
        phi = rng.uniform(0.0, 2.0 * np.pi, size=(3, 2))
        tp = 2.0 * np.pi
        X0, Y0, Z0 = X, Y, Z
        X = X0 + deform * np.sin(tp * Y0 + phi[0, 0]) * np.sin(tp * Z0 + phi[0, 1])
        Y = Y0 + deform * np.sin(tp * Z0 + phi[1, 0]) * np.sin(tp * X0 + phi[1, 1])
        Z = Z0 + deform * np.sin(tp * X0 + phi[2, 0]) * np.sin(tp * Y0 + phi[2, 1])

    gx, gy = nx * N + 1, ny * N + 1
    gid = (I + gx * (J + gy * K)).astype(np.int64)
    if dirichlet:
        bnd = ((I == 0) | (I == nx * N) | (J == 0) | (J == ny * N)
               | (K == 0) | (K == nz * N))
        dmask = bnd.astype(np.uint8)
    else:
        dmask = np.zeros((E, NP, NP, NP), dtype=np.uint8)

    def flat(a, dt):
        return np.ascontiguousarray(np.asarray(a, dtype=dt).reshape(E, NP ** 3))

    return BoxMesh(N=N, shape=(nx, ny, nz), x=flat(X, np.float64), y=flat(Y, np.float64),
                   z=flat(Z, np.float64), gid=flat(gid, np.int64),
                   dirichlet=flat(dmask, np.uint8), deform=deform, seed=seed)


def relabel(mesh: BoxMesh, seed: int) -> BoxMesh:
    """Same geometry with elements permuted and global IDs randomly renumbered.

    Used to check that nothing depends on lattice ordering of elements or IDs.
    Returns the permuted mesh; mesh.meta["perm"] holds the element permutation
    (new element e is old element perm[e]).
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(mesh.E)
    ids, inv = np.unique(mesh.gid, return_inverse=True)
    newid = rng.permutation(len(ids)).astype(np.int64) * 3 + 7  # sparse, unordered IDs
    gid = newid[inv.reshape(mesh.gid.shape)]
    out = BoxMesh(N=mesh.N, shape=mesh.shape, x=np.ascontiguousarray(mesh.x[perm]),
                  y=np.ascontiguousarray(mesh.y[perm]), z=np.ascontiguousarray(mesh.z[perm]),
                  gid=np.ascontiguousarray(gid[perm]),
                  dirichlet=np.ascontiguousarray(mesh.dirichlet[perm]),
                  deform=mesh.deform, seed=mesh.seed, meta={"perm": perm})
    return out


def rotate_elements(mesh: BoxMesh, seed: int) -> BoxMesh:
    """Same mesh with each element's local (i, j, k) numbering turned by a
    random proper rotation of the reference cube (24 choices: an even or odd
    axis permutation combined with reflections so the orientation is kept).

    Neighbouring elements then meet with every relative face orientation,
    as in unstructured hex meshes. mesh.meta["rot"] holds the choice per element.
    """
    N = mesh.N
    n = N + 1
    rng = np.random.default_rng(seed)
    idx = np.arange(n ** 3).reshape(n, n, n)  # [k, j, i] -> p
    rots = []
    for perm in ((0, 1, 2), (1, 2, 0), (2, 0, 1), (0, 2, 1), (2, 1, 0), (1, 0, 2)):
        odd = perm in ((0, 2, 1), (2, 1, 0), (1, 0, 2))
        for flips in ((0, 0, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 1)):
            if (sum(flips) % 2 == 1) != odd:
                continue  # keep det = +1
            a = idx.transpose(2, 1, 0)  # [i, j, k]
            a = np.transpose(a, perm)
            for ax, fl in enumerate(flips):
                if fl:
                    a = np.flip(a, axis=ax)
            rots.append(np.ascontiguousarray(a.transpose(2, 1, 0)).ravel())
    choice = rng.integers(0, len(rots), size=mesh.E)
    src = np.stack([rots[c] for c in choice])  # new local p <- old local src[e, p]

    def take(a):
        return np.ascontiguousarray(np.take_along_axis(a, src, axis=1))

    return BoxMesh(N=N, shape=mesh.shape, x=take(mesh.x), y=take(mesh.y), z=take(mesh.z), gid=take(mesh.gid),
                   dirichlet=take(mesh.dirichlet), deform=mesh.deform, seed=mesh.seed, meta={"rot": choice})


def random_rhs(mesh: BoxMesh, seed: int) -> np.ndarray:
    """Consistent, masked random right-hand side, uniform in [-1, 1].

    One value per unique global ID, drawn in ascending ID order from
    default_rng(seed), copied to every local copy, zero on Dirichlet nodes.
    """
    ids, inv = np.unique(mesh.gid, return_inverse=True)
    rng = np.random.default_rng(seed)
    vals = rng.uniform(-1.0, 1.0, size=len(ids))
    b = vals[inv.reshape(mesh.gid.shape)]
    b = np.where(mesh.dirichlet != 0, 0.0, b)
    return np.ascontiguousarray(b, dtype=np.float64)


def rhs_sequence_fn(mesh: BoxMesh, *, modes: int = 6, noise: float = 1e-3, dt: float = 0.05,
                    seed: int = 0, device=None):
    """Right-hand sides b^m that vary smoothly in time, as a function m -> b^m.

    b^m = keep * (sum_k cos(omega_k m dt + phi_k) g_k + noise * eta^m), where
    keep is 0 on Dirichlet nodes and 1 elsewhere and
      g_k   = sin(pi a_k1 x + c_k1) sin(pi a_k2 y + c_k2) sin(pi a_k3 z + c_k3),
              a ~ U{1..4}, c ~ U(0, 2 pi): `modes` fixed smooth fields;
      omega_k ~ U(0.5, 2), phi_k ~ U(0, 2 pi);
      eta^m = sin(q_1 x + s_1) sin(q_2 y + s_2) sin(q_3 z + s_3) with
              q ~ U(100, 300), s ~ U(0, 2 pi) drawn afresh for every step from
              default_rng([seed, m]): a rough field outside the smooth span.
    All values are functions of the node coordinates, so every copy of a shared
    node gets the same value (the vector is consistent). This stands in for
    the pressure right-hand sides of successive time steps, which lie close to
    a low-dimensional space. device=None evaluates with numpy; otherwise with
    torch on that device (for large meshes).
    """
    rng = np.random.default_rng(seed)
    omega = rng.uniform(0.5, 2.0, size=modes)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=modes)
    wave = rng.integers(1, 5, size=(modes, 3))
    shift = rng.uniform(0.0, 2.0 * np.pi, size=(modes, 3))
    if device is None:
        sin = np.sin
        X, Y, Z = mesh.x, mesh.y, mesh.z
        keep = (mesh.dirichlet == 0).astype(np.float64)
    else:
        import torch
        sin = torch.sin
        X, Y, Z = (torch.from_numpy(a).to(device) for a in (mesh.x, mesh.y, mesh.z))
        keep = torch.from_numpy(mesh.dirichlet == 0).to(device=device, dtype=torch.float64)

    def field(a, c):
        return sin(a[0] * X + c[0]) * sin(a[1] * Y + c[1]) * sin(a[2] * Z + c[2])

    g = [keep * field(np.pi * wave[k], shift[k]) for k in range(modes)]

    def at(m: int):
        r = np.random.default_rng([seed, m])
        eta = field(r.uniform(100.0, 300.0, size=3), r.uniform(0.0, 2.0 * np.pi, size=3))
        b = noise * keep * eta
        for k in range(modes):
            b = b + float(np.cos(omega[k] * m * dt + phi[k])) * g[k]
        return b

    return at


def rhs_sequence(mesh: BoxMesh, steps: int, *, modes: int = 6, noise: float = 1e-3,
                 dt: float = 0.05, seed: int = 0) -> list:
    """[b^0, .., b^(steps-1)] of rhs_sequence_fn, as numpy arrays."""
    at = rhs_sequence_fn(mesh, modes=modes, noise=noise, dt=dt, seed=seed)
    return [np.ascontiguousarray(at(m)) for m in range(steps)]


def manufactured_solution(mesh: BoxMesh) -> np.ndarray:
    """u = sin(pi x) sin(pi y) sin(pi z) at the nodes (zero on the unit cube's faces)."""
    return np.sin(np.pi * mesh.x) * np.sin(np.pi * mesh.y) * np.sin(np.pi * mesh.z)


def manufactured_neumann_solution(mesh: BoxMesh) -> np.ndarray:
    """u = cos(pi x) cos(pi y) cos(pi z): zero normal derivative on the unit cube's faces."""
    return np.cos(np.pi * mesh.x) * np.cos(np.pi * mesh.y) * np.cos(np.pi * mesh.z)


def manufactured_source(mesh: BoxMesh) -> np.ndarray:
    """f = -lap(u) = 3 pi^2 sin(pi x) sin(pi y) sin(pi z) at the nodes."""
    return 3.0 * np.pi ** 2 * manufactured_solution(mesh)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def config_meshes():
    """The standard workloads, by name: (elements per side, N, deformation, seed)."""
    return {
        "tiny_4x4x4_N7": dict(n=4, N=7, deform=0.0, seed=1000),
        "ax_64x64x64_N7": dict(n=64, N=7, deform=0.05, seed=1001),
        "pmg_48x48x48_N7": dict(n=48, N=7, deform=0.05, seed=1002),
    }


def batched_problem_specs(count: int = 256, seed: int = 3000):
    """Specs for independent problems: m ~ U{2..12} elements per side, N ~ U{5,7,9}."""
    rng = np.random.default_rng(seed)
    m = rng.integers(2, 13, size=count)
    N = rng.choice(np.array([5, 7, 9]), size=count)
    return [dict(n=int(m[k]), N=int(N[k]), deform=0.05, seed=1000 + k) for k in range(count)]


def serving_mesh_sides():
    """16 resident meshes of m^3 elements, m = round(8 + 32 i / 15), i = 0..15."""
    return [int(round(8 + 32 * i / 15)) for i in range(16)]

"""Projection onto prior solutions (oracle, FP64).

Test infrastructure: see the package docstring.

Implementation section, "Projection Is Key": for a sequence of systems
A x^m = b^m with slowly varying b^m, keep an A-orthonormal basis
P_L = [p_1 .. p_L] of earlier solutions. The A-norm best fit of x^m in
span(P_L) is xbar = P_L P_L^T b^m. The reduced problem A dx = b^m - A xbar
is solved by the Krylov solver and x^m = xbar + dx. The space is augmented
with dx after one round of classical Gram-Schmidt in the A-inner product
against P_L, then normalised in the A-norm. Once L reaches L_max the space is
restarted.

Readings where the paper is silent:
* restart: when the space already holds L_max vectors, the solve still uses
  all of them; afterwards the space is replaced by the normalised newest
  solution x^m alone (x^m / |x^m|_A);
* a correction whose A-orthogonal part is negligible,
  |dx - P beta|_A^2 <= drop_tol * |dx|_A^2, is not added (the space would
  lose A-orthonormality);
* the reduced system's stopping test stays relative to |b^m|: the inner
  solver runs with rtol |b^m| / |b^m - A xbar|; if the projected residual
  already meets rtol, dx = 0 and the space is left unchanged.

Everything is written from the definitions: A xbar is applied directly (the
kernel path reuses A p_i), and the A-norm of the Gram-Schmidt remainder is
computed from A applied to it.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class ProjectionSpace:
    L_max: int
    P: list = field(default_factory=list)

    @property
    def L(self) -> int:
        return len(self.P)


def best_fit(space: ProjectionSpace, dot, b):
    """xbar = P P^T b (a sum of L terms, coefficients (p_i, b))."""
    xbar = np.zeros_like(b)
    for p in space.P:
        xbar = xbar + dot(p, b) * p
    return xbar


def augment(space: ProjectionSpace, apply_A, dot, dx, x, drop_tol=1e-12):
    """Add dx to the space (classical Gram-Schmidt in the A-inner product).

    When the space is full it restarts from the newest solution x alone.
    """
    if space.L >= space.L_max:
        xAx = dot(x, apply_A(x))
        space.P = [x / np.sqrt(xAx)] if xAx > 0 else []
        return
    Adx = apply_A(dx)
    dAd = dot(dx, Adx)
    if not dAd > 0:
        return
    betas = [dot(p, Adx) for p in space.P]  # all against the same dx: one reduction
    v = dx.copy()
    for beta, p in zip(betas, space.P):
        v = v - beta * p
    vAv = dot(v, apply_A(v))
    if vAv > drop_tol * dAd:
        space.P.append(v / np.sqrt(vAv))


def solve_projected(space: ProjectionSpace, apply_A, dot, solve, b, rtol, drop_tol=1e-12):
    """One projected solve: returns (x, dx, relres_initial).

    solve(r, rtol) -> dx solves A dx = r to |r - A dx| <= rtol |r|.
    """
    bb = dot(b, b)
    xbar = best_fit(space, dot, b)
    r = b - apply_A(xbar)
    rel0 = np.sqrt(dot(r, r) / bb) if bb > 0 else 0.0
    if bb == 0 or rel0 <= rtol:
        return xbar, np.zeros_like(b), rel0
    dx = solve(r, rtol / rel0)
    x = xbar + dx
    augment(space, apply_A, dot, dx, x, drop_tol)
    return x, dx, rel0

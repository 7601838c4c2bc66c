"""Reference-element operators on Gauss-Lobatto-Legendre (GLL) points (oracle, FP64).

Test infrastructure: see the package docstring.

The SEM represents a field on each element by its values at the tensor grid of
N+1 GLL points per direction, with Lagrange interpolants h_i (Algorithms,
eq. field1). The derivative matrix Dhat_il = h_l'(xi_i) turns differentiation
into a small dense matrix product (Algorithms, footnote to eq. field1). The
p-multigrid interpolation Jhat maps coarse-level GLL values to fine-level GLL
points (Implementation, pMG paragraph).

Textbook definitions used here (Deville, Fischer & Mund 2002, the paper's
reference for the SEM):
  * GLL points: -1, +1 and the N-1 roots of P_N', P_N the Legendre polynomial;
  * GLL weights: w_i = 2 / (N (N+1) P_N(xi_i)^2);
  * Dhat_ij = P_N(xi_i) / (P_N(xi_j) (xi_i - xi_j)) for i != j,
    Dhat_00 = -N(N+1)/4, Dhat_NN = +N(N+1)/4, other diagonal entries 0;
  * Jhat_ij = prod_{k != j} (x_i - y_k) / (y_j - y_k), the j-th Lagrange
    polynomial on the source points y evaluated at target point x_i.
"""
from __future__ import annotations

import numpy as np


def legendre(N: int, x: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(P_N(x), P_{N-1}(x)) by the three-term recurrence
    (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for k in range(1, N):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p, p_prev


def gll(N: int) -> tuple[np.ndarray, np.ndarray]:
    """GLL nodes (ascending) and weights for polynomial order N >= 1.

    The nodes are the zeros of f(x) = x P_N(x) - P_{N-1}(x), which equals
    (x^2 - 1) P_N'(x) / N and so vanishes at +-1 and at the roots of P_N'.
    Its derivative is f'(x) = (N+1) P_N(x), which gives the Newton step
    x <- x - f(x) / ((N+1) P_N(x)), started from the Chebyshev-Gauss-Lobatto
    points -cos(pi i / N).
    """
    if N < 1:
        raise ValueError("N >= 1 required")
    x = -np.cos(np.pi * np.arange(N + 1) / N)
    for _ in range(100):
        p, pm = legendre(N, x)
        dx = (x * p - pm) / ((N + 1) * p)
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    p, _ = legendre(N, x)
    w = 2.0 / (N * (N + 1) * p * p)
    return x, w


def deriv_matrix(N: int) -> np.ndarray:
    """Dhat_ij = h_j'(xi_i) on the GLL points of order N ((N+1) x (N+1))."""
    x, _ = gll(N)
    p, _ = legendre(N, x)
    n = N + 1
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = p[i] / (p[j] * (x[i] - x[j]))
    D[0, 0] = -N * (N + 1) / 4.0
    D[N, N] = N * (N + 1) / 4.0
    return D


def interp_matrix(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """J_ij = h^src_j(dst_i): Lagrange basis on points src evaluated at dst."""
    src = np.asarray(src, dtype=np.float64)
    dst = np.asarray(dst, dtype=np.float64)
    J = np.ones((len(dst), len(src)))
    for i in range(len(dst)):
        for j in range(len(src)):
            for k in range(len(src)):
                if k != j:
                    J[i, j] *= (dst[i] - src[k]) / (src[j] - src[k])
    return J


def prolongation_1d(Nc: int, Nf: int) -> np.ndarray:
    """Jhat from order-Nc GLL values to order-Nf GLL points ((Nf+1) x (Nc+1))."""
    return interp_matrix(gll(Nc)[0], gll(Nf)[0])

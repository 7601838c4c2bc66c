"""Krylov solvers, Chebyshev smoother and power iteration (oracle, FP64).

Test infrastructure: see the package docstring.

All vectors are consistent, masked E-vectors; inner products and norms are
over unique DOFs (operators.dot). Operators are passed as callables v -> A v.

* Jacobi-PCG: the paper solves the velocity Helmholtz systems with
  Jacobi-preconditioned CG (Implementation, Helmholtz paragraph); here it is
  also the FP64 baseline Poisson solver and the coarse-grid solver. Standard
  preconditioned CG (Saad, Iterative Methods, Alg. 9.1), x0 = 0, stop when
  ||r|| / ||b|| <= rtol with the recurrence residual.
* Flexible CG: the outer solver around the (nonsymmetric) pMG preconditioner
  with a short recurrence (Implementation, FlexCG/GMRES paragraph). The
  Polak-Ribiere form beta = (z_new, r_new - r_old) / (z_old, r_old)
  (Notay 2000) is used.
* Flexible GMRES(K): the alternative outer solver (same paragraph; GMRES
  with K bounded by 6 in Performance Results), right-preconditioned so the
  preconditioner may vary between steps.
* Chebyshev acceleration of point Jacobi (Implementation, pMG smoothers;
  Saad, Alg. 12.1) on the interval [lo rho, hi rho] of D^-1 A.
* Power iteration for rho = lambda_max(D^-1 A).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    relres: float
    history: list


def pcg(apply_A, apply_M, dot, b, rtol=1e-8, maxit=10000, fixed_iters=None):
    """Preconditioned CG with x0 = 0.

    fixed_iters: run exactly that many iterations (no convergence test), used
    to compare iterates in parity tests.
    """
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.sqrt(dot(b, b))
    hist = []
    if bnorm == 0.0:
        return SolveResult(x, 0, 0.0, hist)
    z = apply_M(r)
    p = z.copy()
    rz = dot(r, z)
    it = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    relres = 1.0
    while it < limit:
        w = apply_A(p)
        alpha = rz / dot(p, w)
        x = x + alpha * p
        r = r - alpha * w
        it += 1
        relres = np.sqrt(dot(r, r)) / bnorm
        hist.append(relres)
        if fixed_iters is None and relres <= rtol:
            break
        z = apply_M(r)
        rz_new = dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return SolveResult(x, it, relres, hist)


def flexcg(apply_A, apply_M, dot, b, rtol=1e-8, maxit=1000, fixed_iters=None, callback=None):
    """Flexible CG (Polak-Ribiere beta) with x0 = 0.

    callback(k, p, w), if given, sees every search direction p_k and w = A p_k
    (k = 0, 1, ...) as soon as w is formed.
    """
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.sqrt(dot(b, b))
    hist = []
    if bnorm == 0.0:
        return SolveResult(x, 0, 0.0, hist)
    z = apply_M(r)
    p = z.copy()
    rz = dot(r, z)
    it = 0
    limit = fixed_iters if fixed_iters is not None else maxit
    relres = 1.0
    while it < limit:
        w = apply_A(p)
        if callback is not None:
            callback(it, p, w)
        alpha = rz / dot(p, w)
        x = x + alpha * p
        r_old = r
        r = r - alpha * w
        it += 1
        relres = np.sqrt(dot(r, r)) / bnorm
        hist.append(relres)
        if fixed_iters is None and relres <= rtol:
            break
        z = apply_M(r)
        beta = dot(z, r - r_old) / rz
        rz = dot(r, z)
        p = z + beta * p
    return SolveResult(x, it, relres, hist)


def fgmres(apply_A, apply_M, dot, b, K, rtol=1e-8, maxit=1000, fixed_iters=None):
    """Right-preconditioned flexible GMRES(K) with x0 = 0 (Saad 1993).

    Arnoldi on v_0 = b / |b|: z_j = M(v_j), w = A z_j, h_ij = (v_i, w) for
    i <= j (classical Gram-Schmidt: every coefficient against the same w),
    h_{j+1,j} = |w - sum_i h_ij v_i|, v_{j+1} = that vector / h_{j+1,j}.
    The iterate x = x_start + Z y with y minimising |beta e_1 - H y| (a
    library least-squares solve of the (j+2) x (j+1) Hessenberg matrix); that
    minimum is the residual norm used for the stopping test. After K steps the
    method restarts from the true residual b - A x. hist[j] is the relative
    least-squares residual after step j + 1.
    """
    x = np.zeros_like(b)
    bnorm = np.sqrt(dot(b, b))
    hist = []
    if bnorm == 0.0:
        return SolveResult(x, 0, 0.0, hist)
    limit = fixed_iters if fixed_iters is not None else maxit
    it = 0
    r = b.copy()
    relres = 1.0
    while True:
        beta = np.sqrt(dot(r, r))
        V = [r / beta]
        Z = []
        H = np.zeros((K + 1, K))
        y = np.zeros(0)
        stop = False
        for j in range(K):
            Z.append(apply_M(V[j]))
            w = apply_A(Z[j])
            h = [dot(V[i], w) for i in range(j + 1)]
            for i in range(j + 1):
                w = w - h[i] * V[i]
            H[: j + 1, j] = h
            H[j + 1, j] = np.sqrt(dot(w, w))
            V.append(w / H[j + 1, j] if H[j + 1, j] > 0 else w)
            e1 = np.zeros(j + 2)
            e1[0] = beta
            y = np.linalg.lstsq(H[: j + 2, : j + 1], e1, rcond=None)[0]
            relres = np.linalg.norm(e1 - H[: j + 2, : j + 1] @ y) / bnorm
            hist.append(relres)
            it += 1
            if it >= limit or (fixed_iters is None and relres <= rtol) or H[j + 1, j] == 0:
                stop = True
                break
        for i in range(len(y)):
            x = x + y[i] * Z[i]
        if stop:
            break
        r = b - apply_A(x)
    return SolveResult(x, it, relres, hist)


def _precond(dinv, v):
    return dinv(v) if callable(dinv) else dinv * v


def chebyshev(apply_A, dinv, r, rho, degree, lo=0.1, hi=1.1, x0=None):
    """Degree-k Chebyshev-accelerated Jacobi on A x = r, eigen-interval [lo rho, hi rho].

    dinv is the inverse diagonal D^-1 (an array), or any preconditioner given
    as a callable v -> M v (the Chebyshev-accelerated Schwarz smoother), in
    which case D^-1 below reads M.

    theta = (b+a)/2, delta = (b-a)/2, sigma = theta/delta, rho_0 = 1/sigma;
    res = r - A x0; d = D^-1 res / theta; x = x0 + d;
    repeat k-1 times: res -= A d; rho_1 = 1/(2 sigma - rho_0);
                      d = rho_1 rho_0 d + (2 rho_1 / delta) D^-1 res; x += d; rho_0 = rho_1.
    The error after the sweep is p_k(D^-1 A) e0 with
    p_k(l) = T_k((theta - l)/delta) / T_k(theta/delta).
    """
    a, b = lo * rho, hi * rho
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho0 = 1.0 / sigma
    if x0 is None:
        res = r.copy()
        x = np.zeros_like(r)
    else:
        res = r - apply_A(x0)
        x = x0.copy()
    d = _precond(dinv, res) / theta
    x = x + d
    for _ in range(degree - 1):
        res = res - apply_A(d)
        rho1 = 1.0 / (2.0 * sigma - rho0)
        d = rho1 * rho0 * d + (2.0 * rho1 / delta) * _precond(dinv, res)
        x = x + d
        rho0 = rho1
    return x


def power_rho(apply_A, dinv, dot, v0, iters=20):
    """rho ~ lambda_max(D^-1 A) from `iters` normalised power steps.

    v <- D^-1 A v / ||D^-1 A v|| starting from v0 / ||v0||; the estimate is the
    Rayleigh quotient (v, A v) / (v, D v) of the final iterate (D = 1/dinv on
    the unmasked nodes).
    """
    v = v0 / np.sqrt(dot(v0, v0))
    for _ in range(iters):
        v = dinv * apply_A(v)
        v = v / np.sqrt(dot(v, v))
    Av = apply_A(v)
    safe = np.where(dinv != 0, dinv, 1.0)
    Dv = np.where(dinv != 0, v / safe, 0.0)
    return dot(v, Av) / dot(v, Dv)

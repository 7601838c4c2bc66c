"""Pins of the oracle's reference-element operators (GLL, Dhat, Jhat).

Each check is fixed by mathematics, not by the oracle itself: textbook closed
forms (tests/golden/gll_closed_forms.txt), a library root finder, polynomial
exactness of quadrature, differentiation and interpolation.
"""
import os
from math import factorial, sqrt  # noqa: F401  (sqrt is used by the golden expressions)

import numpy as np
import pytest

from oracle import reference_ops as ro
from oracle.counter_rng import splitmix64, start_vector

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gll_closed_forms.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        n, nodes, weights = (s.strip() for s in line.split("|"))
        ev = lambda s: np.array([eval(t, {"sqrt": sqrt}) for t in s.split(",")])  # noqa: E731
        rows.append((int(n), ev(nodes), ev(weights)))
    return rows


@pytest.mark.parametrize("N,nodes,weights", _golden())
def test_gll_closed_forms(N, nodes, weights):
    x, w = ro.gll(N)
    np.testing.assert_allclose(x, nodes, rtol=0, atol=2e-16 * 4)
    np.testing.assert_allclose(w, weights, rtol=4e-15, atol=0)


@pytest.mark.parametrize("N", range(2, 16))
def test_gll_nodes_are_roots_of_legendre_derivative(N):
    # library routine: numpy's Legendre class finds the roots of P_N'
    roots = np.sort(np.polynomial.legendre.Legendre.basis(N).deriv().roots().real)
    x, w = ro.gll(N)
    np.testing.assert_allclose(x[1:-1], roots, atol=1e-13)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert abs(w.sum() - 2.0) < 1e-14


@pytest.mark.parametrize("N", range(1, 13))
def test_gll_quadrature_exactness(N):
    x, w = ro.gll(N)
    for m in range(0, 2 * N):  # exact up to degree 2N-1
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(w, x ** m) - exact) < 1e-13 * max(1, N), (N, m)
    # degree 2N is NOT integrated exactly: the error equals the Lobatto
    # remainder (Abramowitz & Stegun 25.4.32, n = N+1 points, f = x^(2N)):
    # int - sum = -n (n-1)^3 2^(2n-1) ((n-2)!)^4 / ((2n-1) ((2n-2)!)^3) f^(2n-2)
    m = 2 * N
    n = N + 1
    rem = -(n * (n - 1) ** 3 * 2 ** (2 * n - 1) * factorial(n - 2) ** 4
            / ((2 * n - 1) * factorial(2 * n - 2) ** 3)) * factorial(2 * n - 2)
    err = 2.0 / (m + 1) - np.dot(w, x ** m)
    assert abs(err - rem) <= 1e-9 * abs(rem) + 1e-15, (N, err, rem)
    assert abs(err) > 1e-8


@pytest.mark.parametrize("N", range(1, 13))
def test_derivative_matrix(N):
    D = ro.deriv_matrix(N)
    x, _ = ro.gll(N)
    # annihilates constants, differentiates monomials up to degree N exactly
    assert np.max(np.abs(D @ np.ones(N + 1))) < 1e-12 * N * N
    for m in range(1, N + 1):
        np.testing.assert_allclose(D @ x ** m, m * x ** (m - 1), atol=1e-11 * N * N)
    assert D[0, 0] == -N * (N + 1) / 4 and D[N, N] == N * (N + 1) / 4
    if N == 1:
        np.testing.assert_allclose(D, [[-0.5, 0.5], [-0.5, 0.5]], atol=0)


def test_derivative_matrix_vs_barycentric():
    # independent construction: differentiate the barycentric interpolant
    for N in (3, 7, 9):
        x, _ = ro.gll(N)
        n = N + 1
        lam = np.array([1.0 / np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)])
        Db = np.zeros((n, n))
        for i in range(n):
            for j in range(n):
                if i != j:
                    Db[i, j] = lam[j] / lam[i] / (x[i] - x[j])
            Db[i, i] = -Db[i].sum()
        np.testing.assert_allclose(ro.deriv_matrix(N), Db, atol=1e-11 * N * N)


@pytest.mark.parametrize("Nc,Nf", [(1, 3), (3, 7), (2, 5), (4, 9), (1, 7), (6, 8)])
def test_interpolation(Nc, Nf):
    J = ro.prolongation_1d(Nc, Nf)
    assert J.shape == (Nf + 1, Nc + 1)
    np.testing.assert_allclose(J.sum(axis=1), 1.0, atol=1e-13)
    xc, _ = ro.gll(Nc)
    xf, _ = ro.gll(Nf)
    for m in range(Nc + 1):  # exact on polynomials of degree <= Nc
        np.testing.assert_allclose(J @ xc ** m, xf ** m, atol=1e-13)
    # interpolating back to the coarse points is the identity
    Jcf = ro.interp_matrix(xf, xc)
    np.testing.assert_allclose(Jcf @ J, np.eye(Nc + 1), atol=1e-12)
    # endpoint rows are exact unit vectors
    assert np.all(J[0] == np.eye(Nc + 1)[0]) and np.all(J[-1] == np.eye(Nc + 1)[-1])


def test_splitmix64_published_values():
    # reference outputs of splitmix64 for a state initialised to 0:
    # successive calls give 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F
    # (the generator's published test sequence). A call with counter c equals
    # the (c/golden)-th step, so check the first output and the recurrence.
    golden = np.uint64(0x9E3779B97F4A7C15)
    z0 = splitmix64(np.array([0], dtype=np.uint64))[0]
    assert z0 == np.uint64(0xE220A8397B1DCDAF)
    with np.errstate(over="ignore"):
        z1 = splitmix64(np.array([golden], dtype=np.uint64))[0]
        z2 = splitmix64(np.array([golden * np.uint64(2)], dtype=np.uint64))[0]
    assert z1 == np.uint64(0x6E789E6AA1B965F4)
    assert z2 == np.uint64(0x06C45D188009454F)
    v = start_vector(np.arange(100000))
    assert v.min() >= -1 and v.max() < 1 and abs(v.mean()) < 0.01

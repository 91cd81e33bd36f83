"""Pins of the oracle's B-spline basis and 1D Gram matrices (CPU only).

Each check compares the oracle with something other than itself: textbook
identities of B-splines, finite differences, exact rational integration
with sympy's independent B-spline construction, and closed-form interior
rows of the cardinal B-spline Gram matrices.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import bspline, gram


@pytest.mark.parametrize("N,p", [(1, 1), (3, 2), (5, 3), (8, 2), (4, 4)])
def test_partition_of_unity_and_endpoints(N, p):
    knots = bspline.open_uniform_knots(N, p)
    x = np.linspace(0.0, 1.0, 257)
    B = bspline.basis(knots, p, x)
    assert B.shape == (x.size, N + p)
    np.testing.assert_allclose(B.sum(axis=1), 1.0, atol=1e-14)
    assert B.min() >= -1e-15
    assert B[0, 0] == pytest.approx(1.0) and B[-1, -1] == pytest.approx(1.0)
    # open knots: only the first / last function is nonzero at the ends
    assert np.abs(B[0, 1:]).max() < 1e-15 and np.abs(B[-1, :-1]).max() < 1e-15


@pytest.mark.parametrize("N,p", [(3, 1), (4, 2), (6, 3)])
def test_linear_precision_of_greville(N, p):
    """sum_i xi_i B_i(x) = x (textbook identity that defines Greville points)."""
    knots = bspline.open_uniform_knots(N, p)
    x = np.linspace(0.0, 1.0, 101)
    xi = bspline.greville(knots, p)
    np.testing.assert_allclose(bspline.basis(knots, p, x) @ xi, x, atol=1e-14)
    assert xi[0] == 0.0 and xi[-1] == 1.0


@pytest.mark.parametrize("N,p", [(4, 2), (5, 3)])
def test_derivative_matches_finite_difference(N, p):
    knots = bspline.open_uniform_knots(N, p)
    # points away from knots (where derivatives of C^{p-1} splines may jump)
    x = (np.arange(N)[:, None] + np.array([0.13, 0.41, 0.77])[None, :]).ravel() / N
    h = 1e-6
    fd = (bspline.basis(knots, p, x + h) - bspline.basis(knots, p, x - h)) / (2 * h)
    np.testing.assert_allclose(bspline.basis_deriv(knots, p, x), fd, atol=1e-7)


def _sympy_gram(N, p):
    sp = pytest.importorskip("sympy")
    X = sp.Symbol("x")
    knots = [0] * (p + 1) + [sp.Rational(i, N) for i in range(1, N)] + [1] * (p + 1)
    basis = sp.bspline_basis_set(p, knots, X)
    n = N + p
    M = sp.zeros(n, n)
    S = sp.zeros(n, n)
    A = sp.zeros(n, n)
    for e in range(N):
        a, b = sp.Rational(e, N), sp.Rational(e + 1, N)
        mid = (a + b) / 2
        # restrict each piecewise function to the element by evaluating the
        # piece that is active at its midpoint
        loc = []
        for f in basis:
            piece = 0
            for expr, cond in f.args:
                if bool(cond.subs(X, mid)):
                    piece = expr
                    break
            loc.append(sp.expand(piece))
        for l in range(n):
            for i in range(n):
                M[l, i] += sp.integrate(loc[l] * loc[i], (X, a, b))
                S[l, i] += sp.integrate(sp.diff(loc[l], X) * sp.diff(loc[i], X), (X, a, b))
                A[l, i] += sp.integrate(loc[l] * sp.diff(loc[i], X), (X, a, b))
    f = lambda m: np.array(m.tolist(), dtype=float)
    return f(M), f(S), f(A)


@pytest.mark.parametrize("N,p", [(1, 1), (3, 1), (3, 2), (4, 2), (4, 3)])
def test_gram_against_exact_rational_integration(N, p):
    M, S, A, B = gram.gram_matrices(N, p)
    Me, Se, Ae = _sympy_gram(N, p)
    np.testing.assert_allclose(M, Me, atol=1e-14)
    np.testing.assert_allclose(S, Se, atol=1e-11 * N * N)
    np.testing.assert_allclose(A, Ae, atol=1e-13)
    np.testing.assert_array_equal(B, A.T)


# Interior rows on uniform knots (cardinal B-spline autocorrelations),
# offsets -p..p, h = 1/N.
CLOSED_FORM = {
    2: dict(M=[Fraction(c, 120) for c in (1, 26, 66, 26, 1)],
            S=[Fraction(-1, 6), Fraction(-1, 3), Fraction(1), Fraction(-1, 3), Fraction(-1, 6)],
            A=[Fraction(-1, 24), Fraction(-5, 12), 0, Fraction(5, 12), Fraction(1, 24)]),
    3: dict(M=[Fraction(c, 5040) for c in (1, 120, 1191, 2416, 1191, 120, 1)],
            S=[Fraction(-1, 120), Fraction(-1, 5), Fraction(-1, 8), Fraction(2, 3),
               Fraction(-1, 8), Fraction(-1, 5), Fraction(-1, 120)],
            A=[Fraction(-1, 720), Fraction(-7, 90), Fraction(-49, 144), 0, Fraction(49, 144),
               Fraction(7, 90), Fraction(1, 720)]),
}


@pytest.mark.parametrize("p", [2, 3])
@pytest.mark.parametrize("N", [12, 20])
def test_interior_rows_closed_form(N, p):
    M, S, A, _ = gram.gram_matrices(N, p)
    h = 1.0 / N
    i = (N + p) // 2
    cf = CLOSED_FORM[p]
    np.testing.assert_allclose(M[i, i - p:i + p + 1], [float(c) * h for c in cf["M"]], rtol=1e-13)
    np.testing.assert_allclose(S[i, i - p:i + p + 1], [float(c) / h for c in cf["S"]], rtol=1e-12)
    np.testing.assert_allclose(A[i, i - p:i + p + 1], [float(c) for c in cf["A"]], atol=1e-14)


@pytest.mark.parametrize("N,p", [(5, 1), (9, 2), (16, 3)])
def test_gram_sum_rules(N, p):
    M, S, A, _ = gram.gram_matrices(N, p)
    n = N + p
    assert M.sum() == pytest.approx(1.0, abs=1e-13)          # int 1 * 1
    np.testing.assert_allclose(S.sum(axis=1), 0.0, atol=1e-10 * N)  # S 1 = 0
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-13)      # A 1 = int B_l * 0
    col = np.zeros(n)
    col[0], col[-1] = -1.0, 1.0                                     # int B_i' = B_i(1) - B_i(0)
    np.testing.assert_allclose(A.sum(axis=0), col, atol=1e-13)
    np.testing.assert_allclose(M, M.T, atol=1e-16)
    np.testing.assert_allclose(A + A.T, np.outer(np.eye(n)[-1], np.eye(n)[-1])
                               - np.outer(np.eye(n)[0], np.eye(n)[0]), atol=1e-13)
    # banded: bandwidth 2p+1
    iu = np.abs(np.subtract.outer(np.arange(n), np.arange(n))) > p
    assert np.all(M[iu] == 0) and np.all(S[iu] == 0) and np.all(A[iu] == 0)

"""B-spline basis on an open uniform knot vector (oracle, float64).

The paper discretises each axis of the unit cube with degree-p B-splines
of maximal continuity C^{p-1} on a uniform patch (section "Variational
formulation"; the head example uses quadratic C^1 splines; the appendix
shows the open knot vector [0 0 1 2 2] for p = 1).  With N elements the
open uniform knot vector has p+1 repeated zeros, the interior knots i/N,
and p+1 repeated ones, giving n = N + p basis functions.

Basis values follow the Cox-de Boor recursion (textbook definition);
derivatives use the standard degree-lowering identity.
"""
from __future__ import annotations

import numpy as np


def open_uniform_knots(N: int, p: int) -> np.ndarray:
    """Open uniform knot vector on [0, 1] with N elements, degree p."""
    if N < 1 or p < 0:
        raise ValueError("need N >= 1 and p >= 0")
    return np.concatenate([np.zeros(p + 1), np.arange(1, N, dtype=np.float64) / N,
                           np.ones(p + 1)])


def _span_indicator(knots: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Degree-0 B-splines: B_{i,0}(x) = 1 on [t_i, t_{i+1}).

    The right end of the domain is attached to the last non-empty span, so
    that the basis is a partition of unity on the closed interval.
    """
    m = len(knots) - 1
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    B = np.zeros((x.size, m))
    last = max(i for i in range(m) if knots[i + 1] > knots[i])
    for i in range(m):
        a, b = knots[i], knots[i + 1]
        if b <= a:
            continue
        inside = (x >= a) & (x < b)
        if i == last:
            inside |= x == b
        B[:, i] = inside
    return B


def basis(knots: np.ndarray, p: int, x) -> np.ndarray:
    """Values B_{i,p}(x) for all i; shape (len(x), n), n = len(knots) - p - 1."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    B = _span_indicator(knots, x)
    for k in range(1, p + 1):
        m = len(knots) - 1 - k
        Bn = np.zeros((x.size, m))
        for i in range(m):
            d1 = knots[i + k] - knots[i]
            d2 = knots[i + k + 1] - knots[i + 1]
            if d1 > 0:
                Bn[:, i] += (x - knots[i]) / d1 * B[:, i]
            if d2 > 0:
                Bn[:, i] += (knots[i + k + 1] - x) / d2 * B[:, i + 1]
        B = Bn
    return B


def basis_deriv(knots: np.ndarray, p: int, x) -> np.ndarray:
    """First derivatives B'_{i,p}(x); shape (len(x), n).

    B'_{i,p} = p/(t_{i+p}-t_i) B_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1}.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(knots) - p - 1
    if p == 0:
        return np.zeros((x.size, n))
    Bl = basis(knots, p - 1, x)  # n + 1 functions of degree p-1
    D = np.zeros((x.size, n))
    for i in range(n):
        d1 = knots[i + p] - knots[i]
        d2 = knots[i + p + 1] - knots[i + 1]
        if d1 > 0:
            D[:, i] += p / d1 * Bl[:, i]
        if d2 > 0:
            D[:, i] -= p / d2 * Bl[:, i + 1]
    return D


def greville(knots: np.ndarray, p: int) -> np.ndarray:
    """Greville abscissae xi_i = (t_{i+1} + ... + t_{i+p}) / p."""
    n = len(knots) - p - 1
    if p == 0:
        return 0.5 * (knots[:-1] + knots[1:])
    return np.array([knots[i + 1:i + p + 1].sum() / p for i in range(n)])


def gauss_points(N: int, q: int):
    """Gauss-Legendre points and weights on the N uniform elements of [0, 1]."""
    g, w = np.polynomial.legendre.leggauss(q)
    h = 1.0 / N
    pts = (np.arange(N)[:, None] + 0.5 * (g[None, :] + 1.0)) * h
    wts = np.broadcast_to(0.5 * h * w[None, :], pts.shape)
    return pts.ravel(), np.ascontiguousarray(wts).ravel()

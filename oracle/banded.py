"""Banded operators and direction-wise line solves (oracle, float64).

Section "Incorporating non-regular material data ...": the alternating
directions solver turns each 3D Kronecker system into three 1D
multi-diagonal systems with many right-hand sides, solved along x, then y,
then z.  The 1D systems have bandwidth 2p+1 (p sub- and p super-diagonals).

The paper does not say how the banded systems are factorised.  The oracle
uses the textbook Doolittle LU restricted to the band, without pivoting
(every 1D matrix here is a mass matrix plus a non-negative multiple of a
stiffness matrix, symmetric positive definite for constant coefficients);
the tests cross-check it against LAPACK's pivoting banded solver.

Array convention: a field is a NumPy array of shape (nz, ny, nx), x
fastest, so the numpy axis of x is 2, of y is 1 and of z is 0.
"""
from __future__ import annotations

import numpy as np

AXIS = {"x": 2, "y": 1, "z": 0}


def to_band(X: np.ndarray, p: int) -> np.ndarray:
    """Dense n x n matrix -> band array b[i, d] = X[i, i + d - p], d = 0..2p."""
    n = X.shape[0]
    b = np.zeros((n, 2 * p + 1))
    for i in range(n):
        for d in range(2 * p + 1):
            j = i + d - p
            if 0 <= j < n:
                b[i, d] = X[i, j]
    return b


def band_lu(band: np.ndarray, p: int):
    """Pivot-free banded Doolittle LU, vectorised over trailing line axes.

    ``band`` has shape (n, 2p+1, *lines).  Returns (L, U) with
    L[i, k-1] = L_{i, i-k} (k = 1..p) and U[i, d] = U_{i, i+d} (d = 0..p),
    each with the trailing line axes of ``band``.
    """
    n = band.shape[0]
    lines = band.shape[2:]
    L = np.zeros((n, p) + lines)
    U = np.zeros((n, p + 1) + lines)

    def A(i, j):
        return band[i, j - i + p]

    def Lget(i, k):  # L_{i,k}, k < i
        return L[i, i - k - 1]

    def Uget(k, j):  # U_{k,j}, j >= k
        return U[k, j - k]

    for i in range(n):
        for j in range(max(0, i - p), i):
            s = A(i, j).copy()
            for k in range(max(0, i - p), j):
                if j - k <= p:
                    s = s - Lget(i, k) * Uget(k, j)
            L[i, i - j - 1] = s / Uget(j, j)
        for j in range(i, min(n, i + p + 1)):
            s = A(i, j).copy()
            for k in range(max(0, i - p, j - p), i):
                s = s - Lget(i, k) * Uget(k, j)
            U[i, j - i] = s
    return L, U


def band_lu_solve(L: np.ndarray, U: np.ndarray, rhs: np.ndarray, p: int) -> np.ndarray:
    """Forward and backward substitution; rhs has shape (n, *lines)."""
    n = rhs.shape[0]
    y = np.zeros_like(rhs)
    for i in range(n):
        s = rhs[i].copy()
        for k in range(max(0, i - p), i):
            s = s - L[i, i - k - 1] * y[k]
        y[i] = s
    x = np.zeros_like(rhs)
    for i in range(n - 1, -1, -1):
        s = y[i].copy()
        for j in range(i + 1, min(n, i + p + 1)):
            s = s - U[i, j - i] * x[j]
        x[i] = s / U[i, 0]
    return x


def min_pivot_ratio(U: np.ndarray, band: np.ndarray, p: int) -> float:
    """min_i |U_ii| / |A_ii| over all lines (pivot-growth check)."""
    return float(np.min(np.abs(U[:, 0]) / np.abs(band[:, p])))


def _lines(u: np.ndarray, axis: int):
    """Move ``axis`` to the front and flatten the other two axes."""
    v = np.moveaxis(u, axis, 0)
    return v.reshape(v.shape[0], -1), v.shape


def _unlines(w: np.ndarray, shape, axis: int) -> np.ndarray:
    return np.moveaxis(w.reshape(shape), 0, axis)


def solve_axis(u: np.ndarray, axis: int, base: np.ndarray, p: int,
               stiff: np.ndarray | None = None, alpha: np.ndarray | None = None,
               dirichlet: bool = False) -> np.ndarray:
    """Solve the 1D system along ``axis`` for every line of ``u``.

    Each line's matrix is ``base`` (dense n x n), or, when ``alpha`` is
    given, the test-function-wise modified matrix whose row i is
    base[i, :] + alpha[position of row i in this line] * stiff[i, :]
    (eq. dupa1abcdefg and the following equations: each test function's
    row carries its own material).  With ``dirichlet`` the first and last
    rows/columns are identity rows/columns.
    """
    rhs, shape = _lines(u, axis)
    n = rhs.shape[0]
    bb = to_band(base, p)
    if alpha is None:
        band = bb[:, :, None]
    else:
        a, _ = _lines(alpha, axis)
        bs = to_band(stiff, p)
        band = bb[:, :, None] + a[:, None, :] * bs[:, :, None]
    if dirichlet:
        band = band.copy()
        for b in (0, n - 1):
            band[b] = 0.0
            band[b, p] = 1.0
            for d in range(2 * p + 1):  # zero column b in the other rows
                i = b - (d - p)
                if 0 <= i < n and i != b:
                    band[i, d] = 0.0
    # A shared matrix is factorised once (a single line that broadcasts).
    L, U = band_lu(band, p)
    x = band_lu_solve(L, U, rhs, p)
    return _unlines(x, shape, axis)


def apply_axis(u: np.ndarray, X: np.ndarray, axis: int, p: int) -> np.ndarray:
    """out[.., r, ..] = sum_i X[r, i] u[.., i, ..] along ``axis`` (banded)."""
    v, shape = _lines(u, axis)
    n = v.shape[0]
    out = np.zeros_like(v)
    for d in range(-p, p + 1):
        r0, r1 = max(0, -d), min(n, n - d)
        if r1 <= r0:
            continue
        diag = X[np.arange(r0, r1), np.arange(r0, r1) + d]
        out[r0:r1] += diag[:, None] * v[r0 + d:r1 + d]
    return _unlines(out, shape, axis)


def apply3(u: np.ndarray, X: np.ndarray, Y: np.ndarray, Z: np.ndarray, p: int) -> np.ndarray:
    """(X (x) Y (x) Z) u with X acting on x, Y on y and Z on z."""
    return apply_axis(apply_axis(apply_axis(u, Z, 0, p), Y, 1, p), X, 2, p)

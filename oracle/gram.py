"""1D Gram matrices M, S, A, B (oracle, float64).

Section "Variational formulation", definitions after eqs. discrete1-4:
the 3D matrices are Kronecker products of 1D mass matrices M, stiffness
matrices S and advection matrices A and B.  Row index = test function,
column index = trial function:

    M[l, i] = int B_l B_i          S[l, i] = int B_l' B_i'
    A[l, i] = int B_l B_i'         (derivative on the trial function)
    B[l, i] = int B_l' B_i = A[i, l]   (derivative on the test function)

Reading: the paper's sentence describing B says "derivatives in the trial
functions", like A.  That is a misprint: in weak1 the term
(d/dx1 E2, d/dx2 V1) is discretised as A (x) B (x) M, which forces B to
carry the derivative of the *test* function, i.e. B = A^T.

The integrals are evaluated exactly by (p+1)-point Gauss-Legendre
quadrature on every element (the integrands are polynomials of degree at
most 2p on each element).
"""
from __future__ import annotations

import numpy as np

from . import bspline


def gram_matrices(N: int, p: int):
    """Return dense (M, S, A, B) for N uniform elements of degree p."""
    knots = bspline.open_uniform_knots(N, p)
    x, w = bspline.gauss_points(N, p + 1)
    V = bspline.basis(knots, p, x)        # (Q, n)
    D = bspline.basis_deriv(knots, p, x)  # (Q, n)
    M = V.T @ (w[:, None] * V)
    S = D.T @ (w[:, None] * D)
    A = V.T @ (w[:, None] * D)            # rows: test value, cols: trial derivative
    B = A.T.copy()
    return M, S, A, B


def dirichlet(Mat: np.ndarray) -> np.ndarray:
    """Strong homogeneous Dirichlet variant of a 1D solve matrix.

    Row and column 0 and n-1 become identity rows/columns (the paper does not
    say how the PEC conditions are imposed; strong imposition keeps every
    solve banded and of size n).
    """
    out = Mat.copy()
    n = out.shape[0]
    for b in (0, n - 1):
        out[b, :] = 0.0
        out[:, b] = 0.0
        out[b, b] = 1.0
    return out

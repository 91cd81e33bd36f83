"""Manufactured solution and error norms (oracle, float64).

Section "Numerical code verification with manufactured solution": for
eps = mu = 1 on the unit cube the fields u^1, u^2, u^3 (kappa, lambda
nonzero integers) solve Maxwell's equations with PEC boundaries, and
u_A = g u^1_{11} + 2 g u^2_{11} + 3 g u^3_{11} with g = 2/sqrt(14) has unit
L2 norm at t = 0.

Reading: the printed u^2 does not satisfy dH/dt = -curl E; its two magnetic
components have the wrong sign.  With the H part of u^2 negated (H1 = +..,
H3 = -..) all three families are exact solutions (checked symbolically in
the tests).  u^1 and u^3 are used as printed.

The initial state is the L2 projection (Gauss q = p+3 per element) onto
the constrained spline space; errors are absolute L2 and H(curl) norms of
E_h - E and H_h - H by the same quadrature (the paper reports L2 and H-curl
errors of the electric and magnetic fields over t in [0, 1]).
"""
from __future__ import annotations

import numpy as np

from . import banded, bspline, maxwell

GAMMA = 2.0 / np.sqrt(14.0)


def u_family(which: int, kappa: int, lam: int, x, y, z, t, d_dt: bool = False):
    """Six components (E1,E2,E3,H1,H2,H3) of u^which_{kappa,lambda}.

    With ``d_dt`` the time derivative of each component is returned instead
    (E parts carry cos(w t), H parts sin(w t), w = pi sqrt(kappa^2+lambda^2)).
    """
    s = np.sqrt(kappa * kappa + lam * lam)
    w = np.pi * s
    if d_dt:
        C, S = -w * np.sin(w * t), w * np.cos(w * t)
    else:
        C, S = np.cos(w * t), np.sin(w * t)
    pi = np.pi
    zero = np.zeros(np.broadcast(x, y, z).shape)
    if which == 1:
        E1 = np.sin(kappa * pi * y) * np.sin(lam * pi * z) * C
        H2 = -lam / s * np.sin(kappa * pi * y) * np.cos(lam * pi * z) * S
        H3 = kappa / s * np.cos(kappa * pi * y) * np.sin(lam * pi * z) * S
        return [E1 + zero, zero, zero, zero, H2 + zero, H3 + zero]
    if which == 2:
        E2 = np.sin(kappa * pi * x) * np.sin(lam * pi * z) * C
        # sign of the magnetic part corrected (see module docstring)
        H1 = lam / s * np.sin(kappa * pi * x) * np.cos(lam * pi * z) * S
        H3 = -kappa / s * np.cos(kappa * pi * x) * np.sin(lam * pi * z) * S
        return [zero, E2 + zero, zero, H1 + zero, zero, H3 + zero]
    if which == 3:
        E3 = np.sin(kappa * pi * x) * np.sin(lam * pi * y) * C
        H1 = -lam / s * np.sin(kappa * pi * x) * np.cos(lam * pi * y) * S
        H2 = kappa / s * np.cos(kappa * pi * x) * np.sin(lam * pi * y) * S
        return [zero, zero, E3 + zero, H1 + zero, H2 + zero, zero]
    raise ValueError(which)


def u_A(x, y, z, t, d_dt: bool = False):
    """u_A = g u^1_{11} + 2 g u^2_{11} + 3 g u^3_{11}, six components."""
    a = u_family(1, 1, 1, x, y, z, t, d_dt)
    b = u_family(2, 1, 1, x, y, z, t, d_dt)
    c = u_family(3, 1, 1, x, y, z, t, d_dt)
    return [GAMMA * (a[i] + 2.0 * b[i] + 3.0 * c[i]) for i in range(6)]


def curl_u_A(x, y, z, t):
    """curl E and curl H of u_A.

    u_A solves Maxwell's equations with eps = mu = 1 (pinned symbolically in
    the tests), so curl H = dE/dt and curl E = -dH/dt.
    """
    d = u_A(x, y, z, t, d_dt=True)
    return [-d[3], -d[4], -d[5]], [d[0], d[1], d[2]]


class Quadrature:
    """Tensor Gauss quadrature and basis tables for one N (an int, or one
    element count per axis) and p: q points per element and axis."""

    def __init__(self, N, p: int, q: int | None = None):
        self.Ns = maxwell.axis_counts(N)
        self.N, self.p = N, p
        self.q = q if q is not None else p + 3
        self.xs, self.ws, self.Vs, self.Ds = [], [], [], []
        for Na in self.Ns:
            knots = bspline.open_uniform_knots(Na, p)
            x, w = bspline.gauss_points(Na, self.q)
            self.xs.append(x)
            self.ws.append(w)
            self.Vs.append(bspline.basis(knots, p, x))        # (Q_a, n_a)
            self.Ds.append(bspline.basis_deriv(knots, p, x))  # (Q_a, n_a)
        self.x, self.w, self.V, self.D = self.xs[0], self.ws[0], self.Vs[0], self.Ds[0]
        self.Z, self.Y, self.X = np.meshgrid(self.xs[2], self.xs[1], self.xs[0], indexing="ij")
        self.W = np.einsum("k,j,i->kji", self.ws[2], self.ws[1], self.ws[0])

    def evaluate(self, c: np.ndarray, deriv_axis: int | None = None) -> np.ndarray:
        """Spline with coefficients c (nz,ny,nx) at all quadrature points.

        deriv_axis (0=x, 1=y, 2=z) selects a first derivative along that axis.
        """
        T = list(self.Vs)
        if deriv_axis is not None:
            T[deriv_axis] = self.Ds[deriv_axis]
        out = np.einsum("qi,kji->kjq", T[0], c)
        out = np.einsum("qj,kjr->kqr", T[1], out)
        out = np.einsum("qk,kjr->qjr", T[2], out)
        return out

    def l2(self, f: np.ndarray) -> float:
        return float(np.sqrt(np.sum(self.W * f * f)))


def project(prob: maxwell.Problem, quad: Quadrature, values) -> tuple:
    """L2 projection of six component fields (values at quadrature points).

    Solves (M (x) M (x) M) c = (f, V) on the constrained space of each
    component (boundary rows identity, boundary right-hand side zero).
    """
    WV = [V * w[:, None] for V, w in zip(quad.Vs, quad.ws)]  # (Q_a, n_a) per axis
    out = []
    for comp in range(6):
        f = values[comp]
        r = np.einsum("qi,kjq->kji", WV[0], f)
        r = np.einsum("qj,kqi->kji", WV[1], r)
        r = np.einsum("qk,qji->kji", WV[2], r)
        kind, c = ("E", comp) if comp < 3 else ("H", comp - 3)
        dax = maxwell.dirichlet_axes(kind, c)
        r = maxwell.zero_boundary(r, dax)
        u = r
        for a in range(3):
            u = banded.solve_axis(u, maxwell._NP_AXIS[a], prob.axis_ops[a]["M"], prob.p,
                                  dirichlet=a in dax)
        out.append(u)
    return out[0:3], out[3:6]


def mms_initial(prob: maxwell.Problem, quad: Quadrature, t: float = 0.0):
    vals = u_A(quad.X, quad.Y, quad.Z, t)
    return project(prob, quad, vals)


def errors(quad: Quadrature, E, H, t: float):
    """Absolute L2 and H(curl) errors of E and H against u_A at time t."""
    ex = u_A(quad.X, quad.Y, quad.Z, t)
    curlE_ex, curlH_ex = curl_u_A(quad.X, quad.Y, quad.Z, t)
    res = {}
    for name, F, off, curl_ex in (("E", E, 0, curlE_ex), ("H", H, 3, curlH_ex)):
        vals = [quad.evaluate(F[c]) for c in range(3)]
        l2sq = sum(float(np.sum(quad.W * (vals[c] - ex[off + c]) ** 2)) for c in range(3))
        # curl components: (d2 F3 - d3 F2, d3 F1 - d1 F3, d1 F2 - d2 F1)
        cu = [quad.evaluate(F[2], 1) - quad.evaluate(F[1], 2),
              quad.evaluate(F[0], 2) - quad.evaluate(F[2], 0),
              quad.evaluate(F[1], 0) - quad.evaluate(F[0], 1)]
        csq = sum(float(np.sum(quad.W * (cu[c] - curl_ex[c]) ** 2)) for c in range(3))
        res[name + "_L2"] = np.sqrt(l2sq)
        res[name + "_Hcurl"] = np.sqrt(l2sq + csq)
    return res

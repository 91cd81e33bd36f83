"""The two-substep ADI time step for Maxwell's equations (oracle, float64).

Follows, in order:

* section "Alternating directions splitting for Maxwell equations": the
  curl split C1 - C2 and the two-substep scheme (eqs. scheme1a-scheme1d);
* section "Variational formulation": weak forms weak1-weak4 and their
  Kronecker-product discretisation discrete1-discrete4 with the block
  matrices M, K1, K2, R1, R2, C1, C2 built from the 1D factors;
* section "Incorporating non-regular material data ...": eq. dupa1ab (the
  per-component systems), the three direction-wise 1D systems solved along
  x, then y, then z, and the test-function-wise material (eq.
  dupa1abcdefg and the equations after it).

Readings (the paper is silent, ambiguous or misprinted):

R1  Block (3,1) of C2 is printed as M(x)M(x)A; C2's third row is d/dx2 acting
    on the first component (weak2 / weak4 / strong2), i.e. M(x)A(x)M.
R2  discrete4 prints "+ tau/(2 mu) C1 E^{n+1}"; scheme1d / strong4 / weak4 all
    give a minus sign.  The minus sign is used.
R3  Boundary conditions (PEC: E x n = 0, H . n = 0) are imposed strongly:
    E_c vanishes on the faces normal to the two other axes, H_c on the faces
    normal to axis c.  The matching rows/columns of each 1D solve matrix are
    identity rows/columns and the matching right-hand-side rows are zeroed.
R4  Material is attached to test functions (rows): each degree of freedom
    (i,j,k) takes (eps, mu, sigma) of the voxel containing its Greville
    point, see ``sample_material``.
R5  Conductivity and a current source are not in the paper.  They enter as
    eps dE/dt + sigma E = curl H - J with sigma E averaged trapezoidally over
    each half step and J evaluated at the half step's midpoint.  With
    c = sigma tau / (4 eps) every E row is divided by (1 + c):
        alpha = tau^2 / (4 eps mu (1 + c)),  beta = tau / (2 eps (1 + c)),
        gamma = (1 - c) / (1 + c),           delta = tau / (2 mu).
    sigma = 0 gives exactly the coefficients of discrete1-discrete4.
R6  Order of the three 1D solves.  The paper lists the x, then y, then z
    systems and, for a modified row of the second or third system, identifies
    the already-solved (trial) indices with the test indices of the row.  Read
    literally, that solves a product of per-line operators in which the
    coefficient of a y- or z-modified row is taken at a *trial* x (and y)
    index; that operator is not the row-scaled system of eq. dupa1ab and the
    resulting scheme is violently unstable for piecewise-constant material
    (spectral radius 1.3 per step for a two-material half space at
    tau = h/2).  The appendix ("Varying coefficients ...", eq:split1 then
    eq:split2) justifies linear cost by solving the coefficient-carrying
    direction *first* and the unscaled direction afterwards, which is exact.
    The oracle follows the appendix: for every E component the modified axis
    is solved first, then the two remaining axes (shared matrices, which
    commute) in x, y, z order.  The result is exactly the solution of the
    row-scaled global Kronecker system of eq. dupa1ab; the H systems (no
    material on the left) are solved x, then y, then z.
R7  The 1D LU is pivot-free (see ``oracle.banded``).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import banded, bspline, gram

# Right-hand sides of the E systems (dupa1ab; weak1 / weak3).  Each entry is
# (coefficient, sign, source field, operator string XYZ), the operator being
# X (x) Y (x) Z with X acting on x.  Fields: "E1".."E3", "H1".."H3".
E_TERMS = {
    1: (  # substep n -> n+1/2, eq. discrete1
        [("gamma", +1, "E1", "MMM"), ("beta", +1, "H3", "MAM"), ("beta", -1, "H2", "MMA"),
         ("alpha", +1, "E2", "ABM")],
        [("gamma", +1, "E2", "MMM"), ("beta", +1, "H1", "MMA"), ("beta", -1, "H3", "AMM"),
         ("alpha", +1, "E3", "MAB")],
        [("gamma", +1, "E3", "MMM"), ("beta", +1, "H2", "AMM"), ("beta", -1, "H1", "MAM"),
         ("alpha", +1, "E1", "BMA")],
    ),
    2: (  # substep n+1/2 -> n+1, eq. discrete3
        [("gamma", +1, "E1", "MMM"), ("beta", +1, "H3", "MAM"), ("beta", -1, "H2", "MMA"),
         ("alpha", +1, "E3", "AMB")],
        [("gamma", +1, "E2", "MMM"), ("beta", +1, "H1", "MMA"), ("beta", -1, "H3", "AMM"),
         ("alpha", +1, "E1", "BAM")],
        [("gamma", +1, "E3", "MMM"), ("beta", +1, "H2", "AMM"), ("beta", -1, "H1", "MAM"),
         ("alpha", +1, "E2", "MBA")],
    ),
}

# Right-hand sides of the H systems (weak2 / weak4).  Fields with a prime
# ("E1'") are the E components just computed in the same substep.
H_TERMS = {
    1: (  # eq. discrete2
        [("one", +1, "H1", "MMM"), ("delta", -1, "E3", "MAM"), ("delta", +1, "E2'", "MMA")],
        [("one", +1, "H2", "MMM"), ("delta", -1, "E1", "MMA"), ("delta", +1, "E3'", "AMM")],
        [("one", +1, "H3", "MMM"), ("delta", -1, "E2", "AMM"), ("delta", +1, "E1'", "MAM")],
    ),
    2: (  # eq. discrete4 (with the sign of scheme1d, reading R2)
        [("one", +1, "H1", "MMM"), ("delta", +1, "E2", "MMA"), ("delta", -1, "E3'", "MAM")],
        [("one", +1, "H2", "MMM"), ("delta", +1, "E3", "AMM"), ("delta", -1, "E1'", "MMA")],
        [("one", +1, "H3", "MMM"), ("delta", +1, "E1", "MAM"), ("delta", -1, "E2'", "AMM")],
    ),
}

# Axis (0 = x, 1 = y, 2 = z) whose 1D system carries the stiffness term for
# E_c: K1 = diag(MSM, MMS, SMM), K2 = diag(MMS, SMM, MSM).
MOD_AXIS = {1: (1, 2, 0), 2: (2, 0, 1)}

_NP_AXIS = (2, 1, 0)  # x, y, z -> numpy axis of a (nz, ny, nx) array


def dirichlet_axes(kind: str, c: int):
    """Axes (0=x,1=y,2=z) in which component c of E or H is constrained (R3)."""
    if kind == "E":
        return tuple(a for a in range(3) if a != c)
    return (c,)


def zero_boundary(R: np.ndarray, axes: Sequence[int]) -> np.ndarray:
    R = R.copy()
    for a in axes:
        ax = _NP_AXIS[a]
        idx = [slice(None)] * 3
        for b in (0, R.shape[ax] - 1):
            idx[ax] = b
            R[tuple(idx)] = 0.0
    return R


def source_time(t, src) -> float:
    """g(t) = sin(2 pi f0 (t - t0)) exp(-((t - t0)/w)^2) (not in the paper, R5)."""
    s = t - src.t0
    return float(np.sin(2.0 * np.pi * src.f0 * s) * np.exp(-(s / src.width) ** 2))


def voxel_weights(N: int, p: int, V: int) -> np.ndarray:
    """W[i, v] = (integral of B_i over voxel v) / (integral of B_i over [0, 1]).

    Each voxel [v/V, (v+1)/V] is split at the knots inside it and every piece
    is integrated with (p + 1)-point Gauss-Legendre (exact for the degree-p
    pieces)."""
    knots = bspline.open_uniform_knots(N, p)
    n = N + p
    g, w = np.polynomial.legendre.leggauss(p + 1)
    W = np.zeros((n, V))
    inner = np.unique(knots)
    for v in range(V):
        a, b = v / V, (v + 1) / V
        cuts = np.concatenate([[a], inner[(inner > a) & (inner < b)], [b]])
        for lo, hi in zip(cuts[:-1], cuts[1:]):
            x = 0.5 * (lo + hi) + 0.5 * (hi - lo) * g
            W[:, v] += (0.5 * (hi - lo) * w) @ bspline.basis(knots, p, x)
    return W / W.sum(axis=1, keepdims=True)


def axis_counts(N):
    """Elements per axis (Nx, Ny, Nz) of a patch given as N (cubic) or a triple."""
    Ns = tuple(int(v) for v in np.broadcast_to(np.asarray(N), (3,)))
    if min(Ns) < 1:
        raise ValueError("need at least one element per axis")
    return Ns


def average_material(N, p: int, eps_vox, mu_vox, sig_vox):
    """Per-DOF (eps, mu, sigma) as the B-spline-weighted average of a voxel map:
    the material of test function B_r B_s B_t is the mean of the voxel values
    weighted by that function (a smoother alternative to Greville sampling of
    the test-function-wise material of the section on non-regular material).
    Voxel arrays are (Vz, Vy, Vx); N is the element count, or one per axis."""
    Nx, Ny, Nz = axis_counts(N)
    Vz, Vy, Vx = np.shape(eps_vox)
    wx, wy, wz = voxel_weights(Nx, p, Vx), voxel_weights(Ny, p, Vy), voxel_weights(Nz, p, Vz)
    def avg(m):
        m = np.asarray(m, float)                  # (Vz, Vy, Vx)
        m = np.einsum("ia,cba->cbi", wx, m)       # x
        m = np.einsum("jb,cbi->cji", wy, m)       # y
        return np.einsum("kc,cji->kji", wz, m)    # z
    return avg(eps_vox), avg(mu_vox), avg(sig_vox)


def sample_material(N, p: int, eps_vox, mu_vox, sig_vox):
    """Per-DOF (eps, mu, sigma) by Greville sampling of a voxel map (R4).

    Voxel arrays are (Vz, Vy, Vx); DOF (i,j,k) takes the voxel that contains
    (xi_i, xi_j, xi_k), voxel index min(floor(xi * V), V - 1) per axis.  N is
    the element count, or one per axis.
    """
    xi = [bspline.greville(bspline.open_uniform_knots(Na, p), p) for Na in axis_counts(N)]
    Vz, Vy, Vx = np.shape(eps_vox)
    ix = np.minimum(np.floor(xi[0] * Vx).astype(int), Vx - 1)
    iy = np.minimum(np.floor(xi[1] * Vy).astype(int), Vy - 1)
    iz = np.minimum(np.floor(xi[2] * Vz).astype(int), Vz - 1)
    sel = np.ix_(iz, iy, ix)
    return (np.asarray(eps_vox, float)[sel], np.asarray(mu_vox, float)[sel],
            np.asarray(sig_vox, float)[sel])


def coefficients(eps, mu, sig, dt):
    """Per-row coefficients (R5); sigma = 0 reproduces discrete1-discrete4."""
    c = sig * dt / (4.0 * eps)
    alpha = dt * dt / (4.0 * eps * mu * (1.0 + c))
    beta = dt / (2.0 * eps * (1.0 + c))
    gamma = (1.0 - c) / (1.0 + c)
    delta = dt / (2.0 * mu)
    return {"alpha": alpha, "beta": beta, "gamma": gamma, "delta": delta}


@dataclasses.dataclass
class Problem:
    """A patch of Nx x Ny x Nz elements of degree p (N an int for a cube, or
    a triple) with per-DOF material and a step.  Each axis has its own 1D
    matrices; the field arrays are (nz, ny, nx), n_a = N_a + p (the paper's
    reordering of a right-hand side into N_x rows of N_y N_z columns)."""

    N: object
    p: int
    eps: np.ndarray
    mu: np.ndarray
    sig: np.ndarray
    dt: float
    source: Optional[object] = None
    # Local time step per test function (section on non-regular material
    # data: tau may be replaced by tau-hat for test function rst like eps and
    # mu): per-DOF array used in the row coefficients, or None for dt.  The
    # time levels (source time, step count) stay those of dt.
    local_dt: Optional[np.ndarray] = None

    def __post_init__(self):
        self.Ns = axis_counts(self.N)
        self.ns = tuple(Na + self.p for Na in self.Ns)
        self.cubic = len(set(self.Ns)) == 1
        if self.cubic:
            self.N, self.n = self.Ns[0], self.ns[0]
        shape = self.shape = (self.ns[2], self.ns[1], self.ns[0])
        self.eps = np.broadcast_to(np.asarray(self.eps, float), shape).copy()
        self.mu = np.broadcast_to(np.asarray(self.mu, float), shape).copy()
        self.sig = np.broadcast_to(np.asarray(self.sig, float), shape).copy()
        if np.any(self.eps <= 0) or np.any(self.mu <= 0) or np.any(self.sig < 0):
            raise ValueError("need eps > 0, mu > 0, sigma >= 0")
        # per axis (x, y, z): {"M", "S", "A", "B"} of that axis's 1D space
        self.axis_ops = []
        for Na in self.Ns:
            M, S, A, B = gram.gram_matrices(Na, self.p)
            self.axis_ops.append({"M": M, "S": S, "A": A, "B": B})
        self.M, self.S, self.A, self.B = (self.axis_ops[0][k] for k in "MSAB")
        tau = self.dt if self.local_dt is None else \
            np.broadcast_to(np.asarray(self.local_dt, float), shape).copy()
        self.coef = coefficients(self.eps, self.mu, self.sig, tau)
        self.coef["one"] = np.ones(shape)
        self.axis_knots = [bspline.open_uniform_knots(Na, self.p) for Na in self.Ns]
        self.knots = self.axis_knots[0]

    # -- building blocks ---------------------------------------------------
    def apply(self, u: np.ndarray, ops: str) -> np.ndarray:
        """(X (x) Y (x) Z) u for an operator string "XYZ" (each letter the 1D
        matrix of its own axis)."""
        X, Y, Z = (self.axis_ops[a][o] for a, o in enumerate(ops))
        return banded.apply3(u, X, Y, Z, self.p)

    def source_time(self, sub: int, t: float) -> float:
        """Time at which the source of substep ``sub`` starting at t is
        evaluated: the midpoint of the half step (reading R5), t + dt/4 in
        substep 1 and t + 3 dt/4 in substep 2."""
        return t + (0.25 if sub == 1 else 0.75) * self.dt

    def source_rows(self, c: int, t: float) -> np.ndarray:
        """(J(t), V_rst) for component c: a g(t) B_r(xs) B_s(ys) B_t(zs) for
        the point dipole; a source object with its own ``rows`` method
        (e.g. ``SeparableSource``) computes the rows itself."""
        out = np.zeros(self.shape)
        src = self.source
        if src is not None and hasattr(src, "rows"):
            return src.rows(self, c, t)
        if src is None or src.comp != c or src.amp == 0.0:
            return out
        bx, by, bz = (bspline.basis(self.axis_knots[a], self.p, [src.xs[a]])[0] for a in range(3))
        return src.amp * source_time(t, src) * np.einsum("k,j,i->kji", bz, by, bx)

    def solve3(self, R: np.ndarray, kind: str, c: int, mod_axis: Optional[int]) -> np.ndarray:
        """The three 1D solves of component c of E or H (reading R6 for the order).

        With a modified axis the result is (X (x) Y (x) Z)^{-1} R with the
        modified factor's rows carrying the per-test-function coefficient.
        """
        dax = dirichlet_axes(kind, c)
        order = [0, 1, 2] if mod_axis is None else \
            [mod_axis] + [a for a in range(3) if a != mod_axis]
        u = R
        for a in order:
            Ma = self.axis_ops[a]["M"]
            if a == mod_axis:
                u = banded.solve_axis(u, _NP_AXIS[a], Ma, self.p, stiff=self.axis_ops[a]["S"],
                                      alpha=self.coef["alpha"], dirichlet=a in dax)
            else:
                u = banded.solve_axis(u, _NP_AXIS[a], Ma, self.p, dirichlet=a in dax)
        return u

    def rhs_E(self, sub: int, fields: dict, c: int, t_mid: float) -> np.ndarray:
        R = np.zeros(self.shape)
        for coef, sign, f, ops in E_TERMS[sub][c]:
            R += sign * self.coef[coef] * self.apply(fields[f], ops)
        R -= self.coef["beta"] * self.source_rows(c, t_mid)
        return zero_boundary(R, dirichlet_axes("E", c))

    def rhs_H(self, sub: int, fields: dict, c: int) -> np.ndarray:
        R = np.zeros(self.shape)
        for coef, sign, f, ops in H_TERMS[sub][c]:
            R += sign * self.coef[coef] * self.apply(fields[f], ops)
        return zero_boundary(R, dirichlet_axes("H", c))

    def substep(self, sub: int, E, H, t: float):
        """One substep (sub = 1: n -> n+1/2, sub = 2: n+1/2 -> n+1)."""
        fields = {"E1": E[0], "E2": E[1], "E3": E[2], "H1": H[0], "H2": H[1], "H3": H[2]}
        t_mid = self.source_time(sub, t)
        En = []
        for c in range(3):
            R = self.rhs_E(sub, fields, c, t_mid)
            En.append(self.solve3(R, "E", c, MOD_AXIS[sub][c]))
        fields.update({"E1'": En[0], "E2'": En[1], "E3'": En[2]})
        Hn = []
        for c in range(3):
            R = self.rhs_H(sub, fields, c)
            Hn.append(self.solve3(R, "H", c, None))
        return En, Hn

    def step(self, E, H, t: float):
        """One full time step n -> n+1; returns (E, H, t + dt)."""
        E1, H1 = self.substep(1, E, H, t)
        E2, H2 = self.substep(2, E1, H1, t)
        return E2, H2, t + self.dt

    def run(self, E, H, t: float, steps: int):
        for _ in range(steps):
            E, H, t = self.step(E, H, t)
        return E, H, t

    # -- state helpers -------------------------------------------------------
    def constrain(self, E, H):
        """Zero the constrained boundary coefficients of a state (R3)."""
        return ([zero_boundary(E[c], dirichlet_axes("E", c)) for c in range(3)],
                [zero_boundary(H[c], dirichlet_axes("H", c)) for c in range(3)])

    def energy(self, E, H) -> float:
        """Discrete energy sum_c (eps E_c, E_c) + (mu H_c, H_c), row-wise material."""
        e = 0.0
        for c in range(3):
            e += float(np.sum(E[c] * self.eps * self.apply(E[c], "MMM")))
            e += float(np.sum(H[c] * self.mu * self.apply(H[c], "MMM")))
        return e


@dataclasses.dataclass
class SeparableSource:
    """A distributed current J = j(t) fx(x) fy(y) fz(z) e_comp (not in the
    paper; reading R5 fixes where J enters).  Its rows (J(t), V_rst) =
    j(t) (fx, B_r)(fy, B_s)(fz, B_t) are integrated with q Gauss-Legendre
    points per element (the profiles need not be polynomials)."""

    comp: int
    j: object          # callable j(t)
    fx: object         # callables of one coordinate (vectorised)
    fy: object
    fz: object
    q: int = 12

    def rows(self, prob: "Problem", c: int, t: float) -> np.ndarray:
        if c != self.comp:
            return np.zeros(prob.shape)
        ints = []
        for a, f in enumerate((self.fx, self.fy, self.fz)):
            x, w = bspline.gauss_points(prob.Ns[a], self.q)
            V = bspline.basis(prob.axis_knots[a], prob.p, x)   # (Q, n_a)
            ints.append((w * f(x)) @ V)
        return float(self.j(t)) * np.einsum("k,j,i->kji", ints[2], ints[1], ints[0])


def problem_from_voxels(N, p: int, material, dt: float, source=None,
                        mapping: str = "greville") -> Problem:
    """Problem with voxel material (sigma non-dimensional) mapped to the test
    functions by Greville sampling or by the B-spline-weighted average."""
    if mapping == "greville":
        eps, mu, sig = sample_material(N, p, material.eps_r, material.mu_r, material.sigma_nd)
    elif mapping == "bspline_avg":
        eps, mu, sig = average_material(N, p, material.eps_r, material.mu_r, material.sigma_nd)
    else:
        raise ValueError(mapping)
    return Problem(N, p, eps, mu, sig, dt, source)

"""Pins of the oracle against the paper's manufactured-solution results,
the scheme's invariants and the appendix toy problem (CPU only)."""
import json
import os

import numpy as np
import pytest

from oracle import banded, bspline, gram, maxwell, mms
from workloads import random_fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("which", [1, 2, 3])
@pytest.mark.parametrize("kappa,lam", [(1, 1), (2, 1), (1, 3)])
def test_families_solve_maxwell_symbolically(which, kappa, lam):
    """dE/dt = curl H, dH/dt = -curl E (eps = mu = 1) and PEC boundaries."""
    sp = pytest.importorskip("sympy")
    x, y, z, t = sp.symbols("x y z t", real=True)
    s = sp.sqrt(kappa ** 2 + lam ** 2)
    w = sp.pi * s
    C, S = sp.cos(w * t), sp.sin(w * t)
    sn, cs, pi = sp.sin, sp.cos, sp.pi
    if which == 1:
        U = [sn(kappa * pi * y) * sn(lam * pi * z) * C, 0, 0,
             0, -lam / s * sn(kappa * pi * y) * cs(lam * pi * z) * S,
             kappa / s * cs(kappa * pi * y) * sn(lam * pi * z) * S]
    elif which == 2:  # magnetic part with the corrected sign
        U = [0, sn(kappa * pi * x) * sn(lam * pi * z) * C, 0,
             lam / s * sn(kappa * pi * x) * cs(lam * pi * z) * S, 0,
             -kappa / s * cs(kappa * pi * x) * sn(lam * pi * z) * S]
    else:
        U = [0, 0, sn(kappa * pi * x) * sn(lam * pi * y) * C,
             -lam / s * sn(kappa * pi * x) * cs(lam * pi * y) * S,
             kappa / s * cs(kappa * pi * x) * sn(lam * pi * y) * S, 0]
    U = [sp.sympify(u) for u in U]
    X = (x, y, z)

    def curl(F):
        return [sp.diff(F[2], y) - sp.diff(F[1], z), sp.diff(F[0], z) - sp.diff(F[2], x),
                sp.diff(F[1], x) - sp.diff(F[0], y)]

    E, H = U[:3], U[3:]
    for c in range(3):
        assert sp.simplify(sp.diff(E[c], t) - curl(H)[c]) == 0
        assert sp.simplify(sp.diff(H[c], t) + curl(E)[c]) == 0
    # PEC: tangential E and normal H vanish on the faces x_a = 0, 1
    for a in range(3):
        for v in (0, 1):
            for c in range(3):
                if c != a:
                    assert sp.simplify(E[c].subs(X[a], v)) == 0
            assert sp.simplify(H[a].subs(X[a], v)) == 0
    # and the oracle's numeric version agrees with the symbolic one
    pts = np.random.default_rng(0).uniform(0, 1, (4, 5))
    num = mms.u_family(which, kappa, lam, pts[0], pts[1], pts[2], pts[3])
    for c in range(6):
        f = sp.lambdify((x, y, z, t), U[c], "numpy")
        np.testing.assert_allclose(num[c], np.broadcast_to(f(*pts), pts[0].shape), atol=1e-14)


def test_printed_u2_is_not_a_solution():
    """Documents the misprint: u^2 with the printed H signs violates dH/dt = -curl E."""
    sp = pytest.importorskip("sympy")
    x, z, t = sp.symbols("x z t", real=True)
    s = sp.sqrt(2)
    E2 = sp.sin(sp.pi * x) * sp.sin(sp.pi * z) * sp.cos(sp.pi * s * t)
    H1_printed = -1 / s * sp.sin(sp.pi * x) * sp.cos(sp.pi * z) * sp.sin(sp.pi * s * t)
    # (curl E)_1 = -dE2/dz
    assert sp.simplify(sp.diff(H1_printed, t) - sp.diff(E2, z)) != 0


def test_gamma_normalises_uA():
    g = _golden("mms_bounds.json")
    q = mms.Quadrature(8, 2, q=8)
    vals = mms.u_A(q.X, q.Y, q.Z, 0.0)
    norm = np.sqrt(sum(np.sum(q.W * v * v) for v in vals))
    assert norm == pytest.approx(g["norm_uA_t0"], abs=1e-12)
    assert 14.0 / 4.0 * mms.GAMMA ** 2 == pytest.approx(g["gamma_squared_times_14_over_4"])


def _mms_run(N, p, steps, T=1.0, n_checks=None):
    dt = T / steps
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, dt)
    quad = mms.Quadrature(N, p)
    E, H = mms.mms_initial(prob, quad)
    t = 0.0
    worst = {k: v for k, v in mms.errors(quad, E, H, 0.0).items()}
    every = 1 if n_checks is None else max(1, steps // n_checks) if n_checks else steps + 1
    for s in range(steps):
        E, H, t = prob.step(E, H, t)
        if (s + 1) % every == 0:
            for k, v in mms.errors(quad, E, H, t).items():
                worst[k] = max(worst[k], v)
    final = mms.errors(quad, E, H, t)
    return worst, final


def test_mms_error_bound_tau_1_10():
    g = _golden("mms_bounds.json")
    worst, _ = _mms_run(g["mesh_elements"], 2, 10)
    assert worst["E_L2"] < g["L2_error_bound"]["10"] and worst["H_L2"] < g["L2_error_bound"]["10"]
    assert worst["E_Hcurl"] < g["Hcurl_error_bound"]["10"]
    assert worst["H_Hcurl"] < g["Hcurl_error_bound"]["10"]


@pytest.mark.slow
def test_mms_error_bound_tau_1_1280():
    g = _golden("mms_bounds.json")
    worst, _ = _mms_run(g["mesh_elements"], 2, 1280, n_checks=32)
    assert worst["E_L2"] < g["L2_error_bound"]["1280"] and worst["H_L2"] < g["L2_error_bound"]["1280"]
    assert worst["E_Hcurl"] < g["Hcurl_error_bound"]["1280"]
    assert worst["H_Hcurl"] < g["Hcurl_error_bound"]["1280"]


def test_second_order_in_time():
    """Errors at T = 1 for tau = 1/10 .. 1/80 on 16^3 p = 2 fall like tau^2."""
    errs = []
    taus = [10, 20, 40]
    for steps in taus:
        _, final = _mms_run(16, 2, steps, n_checks=0)
        errs.append(final["E_L2"] + final["H_L2"])
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.8), rates


def test_spatial_convergence_in_h_and_p():
    """With a tiny time step the error falls at least like h^p (expected h^(p+1))."""
    T = 1.0 / 16.0
    res = {}
    for p in (2, 3):
        for N in (4, 8):
            steps = int(np.ceil(T / (0.25 / N ** 2)))
            _, final = _mms_run(N, p, steps, T=T, n_checks=0)
            res[(N, p)] = final["E_L2"] + final["H_L2"]
    for p in (2, 3):
        rate = np.log2(res[(4, p)] / res[(8, p)])
        assert rate > p, (p, rate)
    assert res[(8, 3)] < res[(8, 2)]


def test_zero_time_step_is_identity():
    N, p = 3, 2
    n = N + p
    prob = maxwell.Problem(N, p, 2.0, 1.5, 0.0, 0.0)
    F = random_fields(n, 11)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    E1, H1, _ = prob.step(E, H, 0.0)
    for a, b in zip(E + H, E1 + H1):
        np.testing.assert_allclose(b, a, atol=1e-13)


def test_linearity():
    N, p = 3, 3
    n = N + p
    rng = np.random.default_rng(3)
    prob = maxwell.Problem(N, p, rng.uniform(1, 9, (n,) * 3), rng.uniform(1, 2, (n,) * 3),
                           rng.uniform(0, 5, (n,) * 3), 0.05)
    F, G = random_fields(n, 1), random_fields(n, 2)
    Ea, Ha = prob.constrain(list(F[:3]), list(F[3:]))
    Eb, Hb = prob.constrain(list(G[:3]), list(G[3:]))
    a, b = 0.7, -1.9
    Ec = [a * u + b * v for u, v in zip(Ea, Eb)]
    Hc = [a * u + b * v for u, v in zip(Ha, Hb)]
    r1 = prob.step(Ea, Ha, 0.0)
    r2 = prob.step(Eb, Hb, 0.0)
    r3 = prob.step(Ec, Hc, 0.0)
    for f in range(2):  # E, H
        for j in range(3):
            np.testing.assert_allclose(r3[f][j], a * r1[f][j] + b * r2[f][j], atol=1e-11)


def _rot(u):
    """Cyclic relabelling x -> y -> z -> x of one scalar coefficient array."""
    return u.transpose(1, 2, 0)


def test_cyclic_equivariance_constant_material():
    """The splitting C1 - C2 is invariant under (x,y,z) -> (y,z,x) with
    (E1,E2,E3) -> (E2,E3,E1): rotating the state commutes with the step."""
    N, p = 3, 2
    n = N + p
    prob = maxwell.Problem(N, p, 3.0, 1.7, 2.0, 0.08)
    F = random_fields(n, 4)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    rotE = lambda E: [_rot(E[2]), _rot(E[0]), _rot(E[1])]
    E1, H1, _ = prob.step(E, H, 0.0)
    E2, H2, _ = prob.step(rotE(E), rotE(H), 0.0)
    for a, b in zip(rotE(E1) + rotE(H1), E2 + H2):
        np.testing.assert_allclose(b, a, atol=1e-12)


def test_cyclic_equivariance_non_cubic_patch():
    """On a patch of Nx x Ny x Nz elements the relabelling x -> y -> z -> x
    turns it into a patch of Nz x Nx x Ny elements: stepping and rotating
    commute with varying material too (each axis keeps its own 1D matrices;
    a mix-up of two axes' matrices breaks this)."""
    Ns, p = (2, 3, 4), 2
    shape = (Ns[2] + p, Ns[1] + p, Ns[0] + p)
    rng = np.random.default_rng(12)
    eps, mu, sig = rng.uniform(1, 20, shape), rng.uniform(0.5, 2, shape), rng.uniform(0, 5, shape)
    prob = maxwell.Problem(Ns, p, eps, mu, sig, 0.07)
    rot = maxwell.Problem((Ns[2], Ns[0], Ns[1]), p, _rot(eps), _rot(mu), _rot(sig), 0.07)
    F = rng.standard_normal((6,) + shape)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    rotE = lambda E: [_rot(E[2]), _rot(E[0]), _rot(E[1])]
    E1, H1, _ = prob.step(E, H, 0.0)
    E2, H2, _ = rot.step(rotE(E), rotE(H), 0.0)
    for a, b in zip(rotE(E1) + rotE(H1), E2 + H2):
        np.testing.assert_allclose(b, a, atol=1e-12 * np.abs(a).max())


def _step_matrix(prob):
    """Dense matrix of one step on the constrained state space (J = 0)."""
    n = prob.n
    D = n ** 3
    cols = []
    for col in range(6 * D):
        v = np.zeros(6 * D)
        v[col] = 1.0
        F = v.reshape(6, n, n, n)
        E, H = prob.constrain(list(F[:3]), list(F[3:]))
        E1, H1, _ = prob.step(E, H, 0.0)
        cols.append(np.concatenate([x.ravel() for x in E1 + H1]))
    return np.array(cols).T


def _half_space(N, p):
    xi = bspline.greville(bspline.open_uniform_knots(N, p), p)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    return np.where(X < 0.5, 1.0, 50.0)


@pytest.mark.parametrize("tau_over_h", [0.5, 10.0, 100.0])
def test_unconditional_stability_constant_material(tau_over_h):
    """Spectral radius of the step map is 1 and its powers stay bounded for any
    tau (the scheme's stated unconditional stability)."""
    N, p = 3, 2
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, tau_over_h / N)
    G = _step_matrix(prob)
    rho = np.abs(np.linalg.eigvals(G)).max()
    assert rho <= 1.0 + 1e-12
    # bounded powers: no growth from 1000 to 4000 steps (the transient bound
    # itself grows with tau / h because the step is a contraction only in a
    # tau-dependent modified norm)
    G1000 = np.linalg.matrix_power(G, 1000)
    G4000 = np.linalg.matrix_power(G1000, 4)
    assert np.linalg.norm(G4000, 2) <= 1.5 * np.linalg.norm(G1000, 2) + 1.0


def test_stability_piecewise_constant_material():
    """eps jumping 1 <-> 50 (a two-material half space) at tau = h/2."""
    N, p = 4, 2
    prob = maxwell.Problem(N, p, _half_space(N, p), 1.0, 0.0, 0.5 / N)
    rho = np.abs(np.linalg.eigvals(_step_matrix(prob))).max()
    assert rho <= 1.0 + 1e-12


def test_literal_sweep_order_is_unstable():
    """Documents reading R6: the x, then y, then z order with the coefficient of
    a modified row read at trial positions is unstable on the same problem."""

    class Literal(maxwell.Problem):
        def solve3(self, R, kind, c, mod_axis):
            dax = maxwell.dirichlet_axes(kind, c)
            u = R
            for a in range(3):
                kw = dict(stiff=self.S, alpha=self.coef["alpha"]) if a == mod_axis else {}
                u = banded.solve_axis(u, maxwell._NP_AXIS[a], self.M, self.p,
                                      dirichlet=a in dax, **kw)
            return u

    N, p = 4, 2
    prob = Literal(N, p, _half_space(N, p), 1.0, 0.0, 0.5 / N)
    rho = np.abs(np.linalg.eigvals(_step_matrix(prob))).max()
    assert rho > 1.1


def test_conductivity_dissipates_energy():
    N, p = 5, 2
    prob = maxwell.Problem(N, p, 1.0, 1.0, 5.0, 0.05)
    quad = mms.Quadrature(N, p)
    E, H = mms.mms_initial(prob, quad)
    e0 = prob.energy(E, H)
    t = 0.0
    for _ in range(40):
        E, H, t = prob.step(E, H, t)
    assert prob.energy(E, H) < 0.5 * e0


def test_appendix_toy_two_stage_solve():
    """Linear B-splines on [0 0 1 2 2]^2 with one eps per test function:
    the oracle's two-stage solve (eq:split1: per-line row-scaled systems
    along x, then eq:split2: the shared mass matrix along y) equals the 9x9
    dense solve of the row-scaled Kronecker system assembled here from
    plain Gauss quadrature."""
    g = _golden("appendix_toy.json")
    knots = np.array(g["knots"], float)
    p = g["degree"]
    n = g["n_per_axis"]
    xq, wq = np.polynomial.legendre.leggauss(2)
    pts = np.concatenate([(e + 0.5 * (xq + 1)) for e in range(2)])
    wts = np.concatenate([0.5 * wq for _ in range(2)])
    V = bspline.basis(knots, p, pts)
    Mx = V.T @ (wts[:, None] * V)
    assert Mx.shape == (n, n)
    # The oracle's Gram matrix lives on [0, 1]: twice it is the mass matrix
    # on [0, 2] (two unit elements).
    M01 = gram.gram_matrices(2, p)[0]
    np.testing.assert_allclose(2.0 * M01, Mx, rtol=1e-14, atol=1e-15)
    rng = np.random.default_rng(9)
    eps = rng.uniform(1, 10, (n, n))  # eps[r, s]: test function B_r(x) B_s(y)
    F = rng.standard_normal((n, n))   # F[r, s] = (F, B_r B_s)
    # global system: row (r,s): sum_{i,j} eps_rs Mx[r,i] My[s,j] u_ij
    G = np.zeros((n * n, n * n))
    for r in range(n):
        for s in range(n):
            for i in range(n):
                for j in range(n):
                    G[r * n + s, i * n + j] = eps[r, s] * Mx[r, i] * Mx[s, j]
    u_dense = np.linalg.solve(G, F.ravel()).reshape(n, n)
    # Stage 1: line s along x solves diag(eps[:, s]) Mx (rows scaled, the
    # base matrix zero); stage 2: the unmodified Mx along y.
    stage1 = banded.solve_axis(F, 0, np.zeros((n, n)), p, stiff=Mx, alpha=eps)
    U = banded.solve_axis(stage1, 1, Mx, p)
    np.testing.assert_allclose(U, u_dense, rtol=1e-13, atol=1e-14)
    # The literal order (shared matrix first) is a different operator.
    W = banded.solve_axis(banded.solve_axis(F, 1, Mx, p), 0, np.zeros((n, n)), p,
                          stiff=Mx, alpha=eps)
    assert np.max(np.abs(W - u_dense)) > 1e-3 * np.max(np.abs(u_dense))


def test_pivot_free_lu_on_strong_material_jump():
    """eps jumping 1 <-> 50 at tau = h/2: no-pivot LU growth stays small."""
    N, p = 32, 3
    M, S, _, _ = gram.gram_matrices(N, p)
    n = N + p
    eps = np.where(np.arange(n) < n // 2, 1.0, 50.0)
    tau = 0.5 / N
    alpha = tau * tau / (4 * eps)
    band = banded.to_band(M, p)[:, :, None] + alpha[:, None, None] * banded.to_band(S, p)[:, :, None]
    L, U = banded.band_lu(band, p)
    assert banded.min_pivot_ratio(U, band, p) > 0.5
    assert np.abs(L).max() < 1.0


def _shell(N, p):
    """Nested boxes around the centre: 1 | 15 | 50 (air, skull-like shell,
    tissue-like core), at the Greville points."""
    xi = bspline.greville(bspline.open_uniform_knots(N, p), p)
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    r = np.maximum(np.maximum(np.abs(X - 0.5), np.abs(Y - 0.5)), np.abs(Z - 0.5))
    return np.where(r < 0.2, 50.0, np.where(r < 0.34, 15.0, 1.0))


@pytest.mark.slow
def test_stability_range_with_material_jumps():
    """The scheme's stability with test-function-wise material, mapped by the
    spectral radius of the step matrix (sigma = 0, J = 0; shell-like 1 | 15 |
    50 jumps, 4^3 elements, p = 2): no growth up to tau = 2h (the coarse step
    of the learned closure), growth at tau = 4h.  With constant material the
    scheme is unconditionally stable (test above); the paper's claim does not
    carry over to per-row material at every step size."""
    N, p = 4, 2
    eps = _shell(N, p)
    for tau_over_h, stable in ((1.0, True), (2.0, True), (4.0, False)):
        prob = maxwell.Problem(N, p, eps, 1.0, 0.0, tau_over_h / N)
        rho = np.abs(np.linalg.eigvals(_step_matrix(prob))).max()
        if stable:
            assert rho <= 1.0 + 1e-12, (tau_over_h, rho)
        else:
            assert rho > 1.0 + 1e-3, (tau_over_h, rho)

"""Pins of the oracle's banded LU, direction sweeps and full ADI step (CPU).

The direction-wise solves are checked against dense Kronecker-product
solves on tiny grids; the full step (constant material, with conductivity
and a point source) against a dense solve of the block systems of eqs.
discrete1-discrete4 assembled directly from the paper's block-matrix list
(with the two misprints fixed as the oracle documents).
"""
import numpy as np
import pytest
from scipy.linalg import solve_banded

from oracle import banded, bspline, gram, maxwell
from workloads import DipoleSource, random_fields


def kron3(X, Y, Z):
    """Dense matrix of X (x) Y (x) Z on the [z][y][x] (x fastest) layout."""
    return np.kron(Z, np.kron(Y, X))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_band_lu_against_lapack(p):
    rng = np.random.default_rng(0)
    n = 23
    A = np.zeros((n, n))
    for d in range(-p, p + 1):
        A += np.diag(rng.uniform(-1, 1, n - abs(d)), d)
    A += np.diag(np.full(n, 2.0 * p + 2.0))
    b = rng.standard_normal((n, 4))
    L, U = banded.band_lu(banded.to_band(A, p)[:, :, None], p)
    x = banded.band_lu_solve(L, U, b, p)
    ab = np.zeros((2 * p + 1, n))
    for i in range(n):
        for j in range(max(0, i - p), min(n, i + p + 1)):
            ab[p + i - j, j] = A[i, j]
    np.testing.assert_allclose(x, solve_banded((p, p), ab, b), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(A @ x, b, atol=1e-12)


@pytest.mark.parametrize("N,p", [(3, 2), (2, 3), (4, 1)])
def test_constant_sweeps_equal_dense_kronecker_solve(N, p):
    """solve[X,Y,Z] = (kron(Z, kron(Y, X)))^-1 rhs for shared 1D matrices."""
    M, S, A, B = gram.gram_matrices(N, p)
    n = N + p
    rng = np.random.default_rng(1)
    X = M + 0.3 * S
    Y = gram.dirichlet(M)
    Z = gram.dirichlet(M + 0.1 * S)
    rhs = maxwell.zero_boundary(rng.standard_normal((n, n, n)), [1, 2])  # y, z constrained
    u = rhs
    u = banded.solve_axis(u, 2, M, p, stiff=S, alpha=np.full((n, n, n), 0.3))
    u = banded.solve_axis(u, 1, M, p, dirichlet=True)
    u = banded.solve_axis(u, 0, M, p, stiff=S, alpha=np.full((n, n, n), 0.1), dirichlet=True)
    ref = np.linalg.solve(kron3(X, Y, Z), rhs.ravel()).reshape(n, n, n)
    np.testing.assert_allclose(u, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("Ns", [(3, 3, 3), (2, 3, 4)])
@pytest.mark.parametrize("c,sub", [(0, 1), (1, 1), (2, 1), (0, 2), (1, 2), (2, 2)])
def test_modified_solve_equals_dense_row_scaled_kronecker(c, sub, Ns):
    """Varying material: the E_c solve equals the dense solve of the row-scaled
    global system of eq. dupa1ab, M..(M + diag(alpha) S)..M restricted to the
    constrained space (reading R6: the modified axis is solved first); also on
    a patch with a different element count per axis, each axis with its own
    1D matrices."""
    p = 2
    G1 = [gram.gram_matrices(Na, p) for Na in Ns]
    shape = (Ns[2] + p, Ns[1] + p, Ns[0] + p)
    rng = np.random.default_rng(2 + c)
    eps = rng.uniform(1.0, 50.0, shape)
    prob = maxwell.Problem(Ns, p, eps, 1.0, 0.0, 0.2)
    alpha = prob.coef["alpha"]
    mod = maxwell.MOD_AXIS[sub][c]
    rhs = maxwell.zero_boundary(rng.standard_normal(shape), maxwell.dirichlet_axes("E", c))
    u = prob.solve3(rhs, "E", c, mod)
    mats = [G1[a][0] for a in range(3)]
    plain = kron3(*mats)
    mats[mod] = G1[mod][1]
    stiff = kron3(*mats)
    G = plain + alpha.ravel()[:, None] * stiff
    free = _free_mask(shape, "E")[c]
    ref = np.zeros(rhs.size)
    ref[free] = np.linalg.solve(G[np.ix_(free, free)], rhs.ravel()[free])
    np.testing.assert_allclose(u.ravel(), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


# ---------------------------------------------------------------------------
# Dense assembly of discrete1-discrete4 straight from the block-matrix list.

def _blocks(G1):
    """Block matrices from the 1D matrices of each axis, G1[a] = (M, S, A, B);
    "XYZ" is X of the x axis (x) Y of the y axis (x) Z of the z axis."""
    idx = {"M": 0, "S": 1, "A": 2, "B": 3}
    k = lambda ops: kron3(*(G1[a][idx[o]] for a, o in enumerate(ops)))
    MMM = k("MMM")
    Z = np.zeros_like(MMM)
    blk = lambda rows: np.block(rows)
    return dict(
        M=blk([[MMM, Z, Z], [Z, MMM, Z], [Z, Z, MMM]]),
        K1=blk([[k("MSM"), Z, Z], [Z, k("MMS"), Z], [Z, Z, k("SMM")]]),
        K2=blk([[k("MMS"), Z, Z], [Z, k("SMM"), Z], [Z, Z, k("MSM")]]),
        R1=blk([[Z, k("ABM"), Z], [Z, Z, k("MAB")], [k("BMA"), Z, Z]]),
        R2=blk([[Z, Z, k("AMB")], [k("BAM"), Z, Z], [Z, k("MBA"), Z]]),
        C1=blk([[Z, Z, k("MAM")], [k("MMA"), Z, Z], [Z, k("AMM"), Z]]),
        # block (3,1) fixed to M (x) A (x) M (reading R1)
        C2=blk([[Z, k("MMA"), Z], [Z, Z, k("AMM")], [k("MAM"), Z, Z]]),
    )


def _free_mask(shape, kind):
    """Per component: boolean mask over the unknowns of E_c or H_c (array
    shape (nz, ny, nx)) that are not constrained."""
    masks = []
    for c in range(3):
        m = np.ones(shape, bool)
        for a in maxwell.dirichlet_axes(kind, c):
            ax = maxwell._NP_AXIS[a]
            idx = [slice(None)] * 3
            for b in (0, shape[ax] - 1):
                idx[ax] = b
                m[tuple(idx)] = False
        masks.append(m.ravel())
    return masks


def _dense_step(N, p, eps, mu, sig, dt, src, E, H, t, tau=None):
    """One step from the dense block systems; eps, mu, sig scalars or per-DOF
    arrays (material attached to test functions = rows, reading R4/R5); tau
    a per-row time step in the row coefficients (default dt)."""
    Ns = maxwell.axis_counts(N)
    shape = (Ns[2] + p, Ns[1] + p, Ns[0] + p)
    D = int(np.prod(shape))
    K = _blocks([gram.gram_matrices(Na, p) for Na in Ns])
    C = K["C1"] - K["C2"]
    full = lambda v: np.tile(np.broadcast_to(np.asarray(v, float), shape).ravel(), 3)
    eps, mu, sig = full(eps), full(mu), full(sig)
    tr = full(dt if tau is None else tau)
    c = sig * tr / (4 * eps)
    a = tr * tr / (4 * eps * mu * (1 + c))
    b = tr / (2 * eps * (1 + c))
    g = (1 - c) / (1 + c)
    d = tr / (2 * mu)
    fe, fh = np.concatenate(_free_mask(shape, "E")), np.concatenate(_free_mask(shape, "H"))

    def J(tt):
        v = np.zeros(3 * D)
        if src is not None:
            bx, by, bz = (bspline.basis(bspline.open_uniform_knots(Ns[a], p), p, [src.xs[a]])[0]
                          for a in range(3))
            g_t = np.sin(2 * np.pi * src.f0 * (tt - src.t0)) * np.exp(-((tt - src.t0) / src.width) ** 2)
            v[src.comp * D:(src.comp + 1) * D] = src.amp * g_t * np.einsum(
                "k,j,i->kji", bz, by, bx).ravel()
        return v

    def solve(Mat, rhs, free):
        x = np.zeros_like(rhs)
        x[free] = np.linalg.solve(Mat[np.ix_(free, free)], rhs[free])
        return x

    e, h = np.concatenate([x.ravel() for x in E]), np.concatenate([x.ravel() for x in H])
    # discrete1 (with conductivity and source, reading R5)
    e1 = solve(K["M"] + a[:, None] * K["K1"], g * (K["M"] @ e) + b * (C @ h)
               + a * (K["R1"] @ e) - b * J(t + dt / 4), fe)
    # discrete2
    h1 = solve(K["M"], K["M"] @ h - d * (K["C1"] @ e) + d * (K["C2"] @ e1), fh)
    # discrete3
    e2 = solve(K["M"] + a[:, None] * K["K2"], g * (K["M"] @ e1) + b * (C @ h1)
               + a * (K["R2"] @ e1) - b * J(t + 3 * dt / 4), fe)
    # discrete4 with the sign of scheme1d (reading R2)
    h2 = solve(K["M"], K["M"] @ h1 + d * (K["C2"] @ e1) - d * (K["C1"] @ e2), fh)
    return ([x.reshape(shape) for x in np.split(e2, 3)], [x.reshape(shape) for x in np.split(h2, 3)])


@pytest.mark.parametrize("N,p,eps,mu,sig,dt,with_src", [
    (2, 2, 1.0, 1.0, 0.0, 0.1, False),
    (3, 2, 2.5, 1.3, 0.0, 0.07, True),
    (2, 3, 4.0, 0.7, 3.0, 0.2, True),
    (3, 1, 1.0, 2.0, 10.0, 0.05, False),
    (3, 2, "rand", "rand", "rand", 0.1, True),
    (2, 3, "rand", 1.0, "rand", 0.3, True),
    ((1, 2, 3), 2, "rand", "rand", "rand", 0.1, True),
    ((3, 1, 2), 3, "rand", 1.0, "rand", 0.2, True),
    ((2, 4, 1), 1, 1.5, 0.8, 2.0, 0.07, True),
])
def test_full_step_equals_dense_block_solve(N, p, eps, mu, sig, dt, with_src):
    """One oracle step against the dense block systems, also on patches with
    a different element count per axis (the paper reorders each right-hand
    side into N_x rows of N_y N_z columns, which allows N_x != N_y != N_z)."""
    Ns = maxwell.axis_counts(N)
    shape = (Ns[2] + p, Ns[1] + p, Ns[0] + p)
    rng = np.random.default_rng(17)
    rnd = lambda v, lo, hi: rng.uniform(lo, hi, shape) if v == "rand" else v
    eps, mu, sig = rnd(eps, 1.0, 50.0), rnd(mu, 0.5, 2.0), rnd(sig, 0.0, 20.0)
    src = DipoleSource(xs=(0.41, 0.55, 0.37), comp=1, amp=0.8, f0=1.5, t0=0.1, width=0.3) \
        if with_src else None
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    F = np.random.default_rng(5).standard_normal((6,) + shape)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    t = 0.03
    E1, H1, t1 = prob.step(E, H, t)
    Ed, Hd = _dense_step(N, p, eps, mu, sig, dt, src, E, H, t)
    for a, b_ in zip(E1 + H1, Ed + Hd):
        np.testing.assert_allclose(a, b_, rtol=1e-11, atol=1e-12 * max(1.0, np.abs(b_).max()))
    assert t1 == pytest.approx(t + dt)


def test_rhs_rows_with_varying_material_equal_dense_row_scaling():
    """E and H right-hand sides with per-row (test function) coefficients."""
    N, p = 3, 2
    n = N + p
    rng = np.random.default_rng(7)
    eps = rng.uniform(1, 50, (n, n, n))
    mu = rng.uniform(0.5, 2, (n, n, n))
    sig = rng.uniform(0, 20, (n, n, n))
    dt = 0.05
    prob = maxwell.Problem(N, p, eps, mu, sig, dt)
    K = _blocks([gram.gram_matrices(N, p)] * 3)
    F = random_fields(n, seed=8)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    e, h = np.concatenate([x.ravel() for x in E]), np.concatenate([x.ravel() for x in H])
    co = prob.coef
    rep = lambda v: np.tile(v.ravel(), 3)
    dense = rep(co["gamma"]) * (K["M"] @ e) + rep(co["beta"]) * ((K["C1"] - K["C2"]) @ h) \
        + rep(co["alpha"]) * (K["R1"] @ e)
    fe = np.concatenate(_free_mask((n, n, n), "E"))
    dense[~fe] = 0.0
    fields = {"E1": E[0], "E2": E[1], "E3": E[2], "H1": H[0], "H2": H[1], "H3": H[2]}
    mine = np.concatenate([prob.rhs_E(1, fields, c, 0.0).ravel() for c in range(3)])
    np.testing.assert_allclose(mine, dense, rtol=1e-12, atol=1e-13 * np.abs(dense).max())


def test_source_rows_partition_of_unity():
    N, p = 6, 3
    src = DipoleSource(xs=(0.3, 0.61, 0.5), comp=2, amp=1.7, f0=2.0, t0=0.0, width=1e9)
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, 0.1, src)
    t = 1.0 / 8.0  # sin(2 pi 2 t) = 1, exp(0) = 1
    rows = prob.source_rows(2, t)
    assert rows.sum() == pytest.approx(1.7, rel=1e-13)
    assert np.count_nonzero(rows) <= (p + 1) ** 3
    assert np.all(prob.source_rows(0, t) == 0)


def test_material_greville_sampling_bruteforce():
    N, p, V = 5, 2, 7
    rng = np.random.default_rng(3)
    vox = rng.uniform(1, 2, (V, V, V))
    eps, _, _ = maxwell.sample_material(N, p, vox, vox, vox)
    knots = bspline.open_uniform_knots(N, p)
    xi = bspline.greville(knots, p)
    n = N + p
    for k in range(n):
        for j in range(n):
            for i in range(n):
                # brute force: first voxel whose box [v/V, (v+1)/V] contains the point
                vi = [next(v for v in range(V) if v / V <= c <= (v + 1) / V and
                           not (c == (v + 1) / V and v + 1 < V))
                      for c in (xi[i], xi[j], xi[k])]
                assert eps[k, j, i] == vox[vi[2], vi[1], vi[0]]


# ------------------------------------------------- B-spline-weighted material
def test_voxel_weights_are_bspline_mass_fractions():
    """W[i, v] against scipy's adaptive quadrature of the oracle basis (a
    different integration method), rows summing to one."""
    from scipy.integrate import quad
    from oracle import bspline
    N, p, V = 5, 3, 7
    W = maxwell.voxel_weights(N, p, V)
    knots = bspline.open_uniform_knots(N, p)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-14)
    for i in (0, 2, N + p - 1):
        f = lambda x: bspline.basis(knots, p, [x])[0, i]
        total = quad(f, 0, 1, points=list(knots[p:-p]), epsabs=1e-14, limit=200)[0]
        # the integral of a B-spline is its knot span over p + 1
        assert total == pytest.approx((knots[i + p + 1] - knots[i]) / (p + 1), rel=1e-12)
        for v in range(V):
            part = quad(f, v / V, (v + 1) / V, points=list(knots[p:-p]), epsabs=1e-14,
                        limit=200)[0]
            assert W[i, v] == pytest.approx(part / total, abs=1e-12)


def test_average_material_constant_and_half_space():
    N, p = 4, 2
    n = N + p
    eps = np.full((6, 5, 8), 3.5)
    e, m, s = maxwell.average_material(N, p, eps, eps * 0 + 1.0, eps * 0)
    assert np.allclose(e, 3.5, rtol=1e-14) and np.allclose(m, 1.0) and np.allclose(s, 0.0)
    # a half space in x (values a | b at x = 1/2): DOF (i, j, k) takes
    # a + (b - a) * (fraction of B_i beyond 1/2), independent of j, k
    a, b = 2.0, 7.0
    vox = np.where((np.arange(8) + 0.5) / 8 > 0.5, b, a)[None, None, :] * np.ones((6, 5, 8))
    e, _, _ = maxwell.average_material(N, p, vox, np.ones_like(vox), np.zeros_like(vox))
    from scipy.integrate import quad
    from oracle import bspline
    knots = bspline.open_uniform_knots(N, p)
    for i in range(n):
        f = lambda x: bspline.basis(knots, p, [x])[0, i]
        frac = quad(f, 0.5, 1, points=list(knots[p:-p]))[0] / quad(f, 0, 1, points=list(knots[p:-p]))[0]
        assert np.allclose(e[:, :, i], a + (b - a) * frac, rtol=1e-10)


# ------------------------------------------------------- local time step
def test_local_time_step_equals_dense_block_solve():
    """Per-test-function tau-hat in every row coefficient (the rst
    modification of the section on non-regular material data) against the
    dense block systems with the same per-row tau."""
    N, p = 3, 2
    n = N + p
    rng = np.random.default_rng(23)
    eps, mu, sig = rng.uniform(1, 30, (n,) * 3), rng.uniform(0.6, 1.8, (n,) * 3), \
        rng.uniform(0, 10, (n,) * 3)
    tau = rng.uniform(0.02, 0.2, (n,) * 3)
    src = DipoleSource(xs=(0.3, 0.6, 0.45), comp=2, amp=1.1, f0=1.5, t0=0.1, width=0.3)
    dt = 0.1
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src, local_dt=tau)
    F = random_fields(n, seed=8)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    E1, H1, t1 = prob.step(E, H, 0.05)
    Ed, Hd = _dense_step(N, p, eps, mu, sig, dt, src, E, H, 0.05, tau=tau)
    for a_, b_ in zip(E1 + H1, Ed + Hd):
        np.testing.assert_allclose(a_, b_, rtol=1e-11, atol=1e-12 * max(1.0, np.abs(b_).max()))
    assert t1 == pytest.approx(0.05 + dt)
    # tau-hat = dt everywhere is the plain step
    plain = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    loc = maxwell.Problem(N, p, eps, mu, sig, dt, src, local_dt=np.full((n,) * 3, dt))
    a1, b1, _ = plain.step(E, H, 0.05)
    a2, b2, _ = loc.step(E, H, 0.05)
    for x, y in zip(a1 + b1, a2 + b2):
        assert np.array_equal(x, y)


def _h_by_line_operators(prob, sub, fields, c):
    """H_c after the H stage written as H_c plus, per curl term of discrete2 /
    discrete4, (+-delta) M_a^{-1} (A_a E_b) along the term's own axis a (the
    mass factors of the two other axes cancelled), with delta taken from the
    first row: valid when delta is one constant."""
    H = fields[f"H{c + 1}"].copy()
    delta = prob.coef["delta"].flat[0]
    for coef, sign, f, ops in maxwell.H_TERMS[sub][c]:
        if coef == "one":
            continue
        a = ops.index("A")
        ax = maxwell._NP_AXIS[a]
        u = banded.apply_axis(fields[f], prob.axis_ops[a]["A"], ax, prob.p)
        H += sign * delta * banded.solve_axis(u, ax, prob.axis_ops[a]["M"], prob.p)
    return H


@pytest.mark.parametrize("N,p", [(4, 2), (5, 3), ((3, 4, 6), 2)])
def test_constant_mu_h_stage_is_one_line_operator_per_term(N, p):
    """With one permeability the H stage's Kronecker solve of each curl term
    reduces to M_a^{-1} A_a along the term's axis, because the constrained
    state vanishes on the faces where the other two mass factors would act
    (the identity the library's H-stage line rounds rest on); with a
    varying permeability it does not."""
    rng = np.random.default_rng(7)
    Ns = maxwell.axis_counts(N)
    shape = (Ns[2] + p, Ns[1] + p, Ns[0] + p)
    eps = rng.uniform(1, 40, shape)
    sig = rng.uniform(0, 5, shape)
    for mu, same in ((1.7, True), (rng.uniform(0.5, 2.0, shape), False)):
        prob = maxwell.Problem(N, p, eps, mu, sig, 0.07)
        F = [rng.standard_normal(shape) for _ in range(9)]
        E, H = prob.constrain(F[0:3], F[3:6])
        En, _ = prob.constrain(F[6:9], F[3:6])
        for sub in (1, 2):
            fields = {"E1": E[0], "E2": E[1], "E3": E[2], "H1": H[0], "H2": H[1], "H3": H[2],
                      "E1'": En[0], "E2'": En[1], "E3'": En[2]}
            for c in range(3):
                full = prob.solve3(prob.rhs_H(sub, fields, c), "H", c, None)
                short = _h_by_line_operators(prob, sub, fields, c)
                err = np.linalg.norm(short - full) / np.linalg.norm(full)
                if same:
                    assert err < 1e-12, (sub, c, err)
                else:
                    assert err > 1e-4, (sub, c, err)

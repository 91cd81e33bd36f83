"""GPU parity: the HIP path (through the C ABI) against the float64 oracle.

Tolerances (relative L2 norm of the difference, per field component):
* float64 path: 1e-12.  Both sides solve the same well-conditioned banded
  systems (1D condition numbers below ~30) in a different summation order,
  so the differences are a few units of roundoff per step.
* float32 mode (float32 state and sweeps, every stage solved in increment
  form from a float64 residual of the old state): 1e-5 per component.  The
  state is stored in float32, which alone (exact solves) adds ~1e-7 of
  relative rounding per step and field; the float32 sweeps act on the
  increments, so their rounding scales with the increments.  The one
  exception is degree 4 from a white-noise state (see its test).
Besides the relative L2 every comparison checks the element-wise largest
difference against the component's largest value, which a localized defect
(a wrong source row, a wrong PEC face) would make of the order of the field
itself: within 1e-12 for float64, within 5e-5 for the float32 mode, whose
rounding errors are spread over all D ~ 10^6 coefficients (the largest of D
such errors exceeds their RMS by about sqrt(2 ln D) ~ 5).
"""
import numpy as np
import pytest

import workloads
from oracle import maxwell, mms

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5
MAXABS_FACTOR32 = 5.0  # element-wise bound of the float32 mode, relative to its L2 bound


@pytest.fixture(scope="module")
def Solver():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_06998_amd.solver import Solver as S
    return S


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def random_setup(N, p, seed, with_src=True, sig_max=20.0):
    n = N + p
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, 50.0, (n, n, n))
    mu = rng.uniform(0.5, 2.0, (n, n, n))
    sig = rng.uniform(0.0, sig_max, (n, n, n))
    src = workloads.DipoleSource(xs=tuple(rng.uniform(0.1, 0.9, 3)), comp=int(seed % 3),
                                 amp=1.3, f0=2.0, t0=0.05, width=0.3) if with_src else None
    return eps, mu, sig, src


def make_gpu(Solver, N, p, eps, mu, sig, dt, src, precision="fp64", res64=None):
    s = Solver(N, p, precision)
    s.set_material_dof(eps, mu, sig)
    if src is not None:
        s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    if res64 is not None:
        s.set_residual64(res64)
    s.factor(dt)
    return s


def constrained_random_state(prob, seed):
    F = workloads.random_fields(prob.n, seed)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    return E, H


def max_abs_rel(a, b):
    """Largest element-wise difference over the largest reference value."""
    m = np.abs(b).max()
    return np.abs(a - b).max() / (m if m > 0 else 1.0)


def compare_state(EH_gpu, E, H, tol, label=""):
    """Per component: relative L2 within tol and element-wise max-abs
    (against the component's largest value) within tol, or within
    MAXABS_FACTOR32 * tol for the float32 mode; a localized error (the source
    rows, a PEC face) cannot hide under the L2 norm."""
    ref = E + H
    errs = [rel_l2(EH_gpu[c], ref[c]) for c in range(6)]
    emax = [max_abs_rel(EH_gpu[c], ref[c]) for c in range(6)]
    tol_max = tol if tol <= TOL64 else MAXABS_FACTOR32 * tol
    assert max(errs) <= tol, (label, "relative L2", errs)
    assert max(emax) <= tol_max, (label, "max-abs", emax)
    return errs


# Up to N = 9 every tile of 8 rows holds a row within 2p of a face; from
# N = 24 on, the middle tiles lie where the y operators' band rows are
# translation-invariant and take their weights from scalar registers, next
# to boundary tiles in the same launch.
@pytest.mark.parametrize("N,p", [(1, 1), (2, 2), (5, 1), (5, 2), (4, 3), (7, 3), (3, 4), (9, 4),
                                 (24, 1), (30, 2), (40, 3), (36, 4)])
@pytest.mark.parametrize("stage,sub", [(0, 1), (0, 2), (1, 1), (1, 2)])
def test_rhs_stage(Solver, N, p, stage, sub):
    eps, mu, sig, src = random_setup(N, p, seed=N * 10 + p)
    dt = 0.07
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, src)
    E, H = constrained_random_state(prob, 3)
    t = 0.2
    if stage == 0:
        fields = {"E1": E[0], "E2": E[1], "E3": E[2], "H1": H[0], "H2": H[1], "H3": H[2]}
        t_mid = t + (0.25 if sub == 1 else 0.75) * dt
        ref = np.stack([prob.rhs_E(sub, fields, c, t_mid) for c in range(3)])
        got = s.rhs(0, sub, np.stack(E + H), t)
    else:
        En, _ = constrained_random_state(prob, 4)
        fields = {"H1": H[0], "H2": H[1], "H3": H[2], "E1": E[0], "E2": E[1], "E3": E[2],
                  "E1'": En[0], "E2'": En[1], "E3'": En[2]}
        ref = np.stack([prob.rhs_H(sub, fields, c) for c in range(3)])
        got = s.rhs(1, sub, np.stack(H + E + En), t)
    for c in range(3):
        assert rel_l2(got[c], ref[c]) <= TOL64, (c, rel_l2(got[c], ref[c]))
        assert max_abs_rel(got[c], ref[c]) <= TOL64, (c, max_abs_rel(got[c], ref[c]))


# n = N + p >= 48 takes the partitioned (4 segments per line) solve for the
# shared-factor axes: n = 48, 54, 59 and 72 cover even and ragged segments
# and every degree; (160, 2) takes the longer register segments (n = 162);
# n >= 193 takes 8 segments per line: (196, 3) ragged (n = 199), (256, 2)
# the lines of the 256^3 workload (n = 258).
@pytest.mark.parametrize("N,p", [(1, 2), (3, 1), (5, 2), (4, 3), (9, 3), (33, 2), (45, 3),
                                 (50, 4), (58, 1), (70, 2)])
@pytest.mark.parametrize("stage,sub", [(0, 1), (0, 2), (1, 1), (1, 2)])
def test_solve_stage(Solver, N, p, stage, sub):
    _solve_stage(Solver, N, p, stage, sub)


@pytest.mark.parametrize("N,p", [(160, 2), (196, 3), (256, 2)])
@pytest.mark.parametrize("stage,sub", [(0, 2), (1, 1)])
def test_solve_stage_long_lines(Solver, N, p, stage, sub):
    _solve_stage(Solver, N, p, stage, sub)


def _solve_stage(Solver, N, p, stage, sub):
    eps, mu, sig, _ = random_setup(N, p, seed=7 + N + p, with_src=False)
    dt = 0.11
    prob = maxwell.Problem(N, p, eps, mu, sig, dt)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, None)
    kind = "E" if stage == 0 else "H"
    rng = np.random.default_rng(5)
    R = [maxwell.zero_boundary(rng.standard_normal((prob.n,) * 3), maxwell.dirichlet_axes(kind, c))
         for c in range(3)]
    ref = [prob.solve3(R[c], kind, c, maxwell.MOD_AXIS[sub][c] if kind == "E" else None)
           for c in range(3)]
    got = s.solve(stage, sub, np.stack(R))
    for c in range(3):
        assert rel_l2(got[c], ref[c]) <= TOL64, (c, rel_l2(got[c], ref[c]))


@pytest.mark.parametrize("N,p,steps", [(1, 1, 3), (2, 3, 3), (3, 2, 4), (6, 2, 3), (5, 3, 3),
                                       (37, 3, 2), (47, 2, 2), (4, 4, 2), (45, 4, 1)])
def test_full_steps_random_material(Solver, N, p, steps):
    eps, mu, sig, src = random_setup(N, p, seed=100 + N)
    dt = 0.5 / N
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, src)
    E, H = constrained_random_state(prob, 9)
    t = 0.01
    s.set_fields(np.stack(E + H), t)
    s.step(steps)
    E, H, t = prob.run(E, H, t, steps)
    got, tg = s.get_fields()
    assert tg == pytest.approx(t, rel=1e-15)
    compare_state(got, E, H, TOL64, (N, p))


@pytest.mark.parametrize("N", [146, 196])
@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32_refine", TOL32)])
def test_large_rounds_two_launches(Solver, precision, tol, N):
    """n = 148: a solve round's x and y/z lines (3 x 343 blocks of 64 lines)
    exceed the single-launch limit of 1024 blocks, so each round runs as two
    concurrent launches joined by events (smaller grids take one mixed-axis
    launch); n = 198 also takes the 8-segment partitioned solve.  One step
    against the oracle."""
    p = 2
    eps, mu, sig, src = random_setup(N, p, seed=7)
    dt = 0.5 / N
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, src, precision)
    E, H = constrained_random_state(prob, 13)
    t = 0.02
    s.set_fields(np.stack(E + H), t)
    s.step(1)
    E, H, t = prob.run(E, H, t, 1)
    got, _ = s.get_fields()
    compare_state(got, E, H, tol, ("n", N + p, precision))


def _fp32_random_steps(Solver, N, p, steps=2, res64=None):
    eps, mu, sig, src = random_setup(N, p, seed=200 + N)
    dt = 0.5 / N
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, src, "fp32_refine", res64)
    E0, H0 = constrained_random_state(prob, 21)
    s.set_fields(np.stack(E0 + H0), 0.01)
    s.step(steps)
    E, H, t = prob.run(E0, H0, 0.01, steps)
    got, tg = s.get_fields()
    assert tg == pytest.approx(t, rel=1e-12)
    return prob, (E0, H0), got, E, H


@pytest.mark.parametrize("N", [4, 45, 128])
def test_full_steps_fp32_refine_random_material(Solver, N):
    """FP32 mode on random per-DOF material from a random (rough) state, two
    steps at p = 3 against the oracle, per component within 1e-5.  n = 48
    and n = 131 run the float32 partitioned sweeps and mixed-axis rounds of
    the 128^3 workload (n = 131 also wraps the ring of per-line factor
    chunks of the material-modified sweeps several times)."""
    _, _, got, E, H = _fp32_random_steps(Solver, N, 3)
    errs = compare_state(got, E, H, TOL32, ("fp32", N, 3))
    print("fp32 random material", N, 3, "errors", errs)


@pytest.mark.parametrize("N", [4, 45])
@pytest.mark.parametrize("res64", [0, 5, 15])
def test_fp32_residual_arithmetic_choices(Solver, N, res64):
    """The float32 mode with its increments formed in float32 arithmetic
    everywhere (0), in float64 for both E stages (5) or for every stage
    (15): all within 1e-5 per component of the oracle at p = 3."""
    _, _, got, E, H = _fp32_random_steps(Solver, N, 3, res64=res64)
    errs = compare_state(got, E, H, TOL32, ("fp32 residual mask", res64, N))
    print("fp32 residual mask", res64, N, "errors", errs)


@pytest.mark.parametrize("N,p,precision,steps", [(45, 3, "fp64", 2), (45, 3, "fp32_refine", 2),
                                                  (62, 2, "fp64", 2), (146, 2, "fp64", 1),
                                                  (196, 2, "fp32_refine", 1), (128, 3, "fp64", 1)])
def test_constant_mu_h_stage_shortcut(Solver, N, p, precision, steps):
    """With one permeability everywhere (delta = dt/(2 mu) the same in every
    row) the H stage runs as two rounds of apply-and-solve lines
    (H_c' = H_c +- delta M_a^-1 A_a E_b per curl term) instead of the
    right-hand side and three mass-solve rounds; random eps and sigma, a
    source, against the oracle's full Kronecker solve.  n = 48 and 64:
    mixed-axis rounds; n = 148: rounds split into concurrent x and y/z
    launches; n = 198: eight segments per line; n = 131: the benchmark's
    lines."""
    eps, _, sig, src = random_setup(N, p, seed=300 + N)
    mu = np.full_like(eps, 1.3)
    dt = 0.5 / N
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, src, precision)
    E, H = constrained_random_state(prob, 23)
    s.set_fields(np.stack(E + H), 0.03)
    s.step(steps)
    E2, H2, t2 = prob.run(E, H, 0.03, steps)
    got, tg = s.get_fields()
    assert tg == pytest.approx(t2, rel=1e-12)
    compare_state(got, E2, H2, TOL64 if precision == "fp64" else TOL32,
                  ("h shortcut", N, p, precision))
    s.profile(1)
    kinds = [L["kind"] for L in s.profile_read()]
    assert "rhs_H" not in kinds and "apply_xyz" in kinds, kinds
    s.close()


class Float32Storage(maxwell.Problem):
    """The oracle with its state rounded to float32 where the float32 mode
    stores it (the E components after the E stage, before the H stage reads
    them; the H components after the H stage), the solves exact: the error
    that float32 storage alone leaves."""

    def substep(self, sub, E, H, t):
        r32 = lambda x: x.astype(np.float32).astype(np.float64)
        fields = {"E1": E[0], "E2": E[1], "E3": E[2], "H1": H[0], "H2": H[1], "H3": H[2]}
        t_mid = self.source_time(sub, t)
        En = [r32(self.solve3(self.rhs_E(sub, fields, c, t_mid), "E", c, maxwell.MOD_AXIS[sub][c]))
              for c in range(3)]
        fields.update({"E1'": En[0], "E2'": En[1], "E3'": En[2]})
        Hn = [r32(self.solve3(self.rhs_H(sub, fields, c), "H", c, None)) for c in range(3)]
        return En, Hn


@pytest.mark.parametrize("N", [4, 45])
def test_full_steps_fp32_refine_degree4_rough(Solver, N):
    """Degree 4 from a white-noise state on random material (sigma up to 20):
    at N = 4 (dt = 1/8) the float32 storage of the state alone, with exact
    solves, leaves up to 1.2e-4 on a strongly damped component, so 1e-5 per
    component is out of reach of any float32-state method there.  The float32
    mode rounds twice per stage (the increment's float32 solve and the stored
    sum), both amplified through the step like the storage rounding: the
    bound per component is 1e-5, or four times the storage-only model's
    error where that is larger (max-abs: MAXABS_FACTOR32 times that)."""
    prob, (E0, H0), got, E, H = _fp32_random_steps(Solver, N, 4)
    S = Float32Storage(prob.N, prob.p, prob.eps, prob.mu, prob.sig, prob.dt, prob.source)
    r32 = lambda L: [x.astype(np.float32).astype(np.float64) for x in L]
    Es, Hs, _ = S.run(r32(E0), r32(H0), 0.01, 2)
    ref = E + H
    model = [rel_l2(a, b) for a, b in zip(Es + Hs, ref)]
    tol = [max(TOL32, 4 * m) for m in model]
    errs = [rel_l2(got[c], ref[c]) for c in range(6)]
    emax = [max_abs_rel(got[c], ref[c]) for c in range(6)]
    print("fp32 degree 4", N, "model", model, "errors", errs, "max-abs", emax)
    assert all(e <= t for e, t in zip(errs, tol)), (errs, tol)
    assert all(e <= MAXABS_FACTOR32 * t for e, t in zip(emax, tol)), (emax, tol)


def test_mms16_manufactured_solution(Solver):
    """16^3 p=2, eps = mu = 1, u_A initial state, 10 steps of 1e-3 (FP64)."""
    w = workloads.make("mms16")
    prob = maxwell.Problem(w.N, w.p, 1.0, 1.0, 0.0, w.dt)
    quad = mms.Quadrature(w.N, w.p)
    E, H = mms.mms_initial(prob, quad)
    s = Solver(w.N, w.p, "fp64")
    s.set_material(w.material.eps_r, w.material.mu_r, w.material.sigma_nd)
    s.factor(w.dt)
    s.set_fields(np.stack(E + H), 0.0)
    s.step(w.steps)
    E, H, t = prob.run(E, H, 0.0, w.steps)
    got, _ = s.get_fields()
    compare_state(got, E, H, TOL64, "mms16")
    err = mms.errors(quad, [got[0], got[1], got[2]], [got[3], got[4], got[5]], t)
    assert err["E_L2"] < 1e-3 and err["H_L2"] < 1e-3


def _workload_pair(Solver, name, steps, precision="fp64", res64=None):
    w = workloads.make(name)
    prob = maxwell.problem_from_voxels(w.N, w.p, w.material, w.dt, w.source)
    s = Solver(w.N, w.p, precision)
    m = w.material
    s.set_material(m.eps_r, m.mu_r, m.sigma_nd)
    src = w.source
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    if res64 is not None:
        s.set_residual64(res64)
    s.factor(w.dt)
    n = w.N + w.p
    # start from a nonzero state so that every term is exercised
    E, H = constrained_random_state(prob, 42)
    E = [1e-3 * e for e in E]
    H = [1e-3 * h for h in H]
    t = 0.45
    s.set_fields(np.stack(E + H), t)
    s.step(steps)
    E, H, t = prob.run(E, H, t, steps)
    got, _ = s.get_fields()
    return got, E, H


def test_blob64_fp64(Solver):
    got, E, H = _workload_pair(Solver, "blob64", 20)
    compare_state(got, E, H, TOL64, "blob64")


def test_blob64_fp32_refine(Solver):
    got, E, H = _workload_pair(Solver, "blob64", 20, "fp32_refine")
    compare_state(got, E, H, TOL32, "blob64 fp32")


def test_shell128_p3_full_size_fp32(Solver):
    """The benchmarked path: the 128^3 p=3 workload in the float32 mode at its
    real size, two steps, every output, per component."""
    got, E, H = _workload_pair(Solver, "shell128", 2, "fp32_refine")
    errs = compare_state(got, E, H, TOL32, "shell128 fp32")
    print("shell128 fp32 per component", errs)


def test_shell128_p3_full_size_fp64(Solver):
    """The 128^3 p=3 workload at its real size: three steps, every output."""
    got, E, H = _workload_pair(Solver, "shell128", 3)
    compare_state(got, E, H, TOL64, "shell128")


def _run_gpu_workload(Solver, name, precision, checkpoints):
    """States of a workload's run from a zero state at the given step counts."""
    w = workloads.make(name)
    s = Solver(w.N, w.p, precision)
    m = w.material
    s.set_material(m.eps_r, m.mu_r, m.sigma_nd)
    src = w.source
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.factor(w.dt)
    n = w.N + w.p
    s.set_fields(np.zeros((6, n, n, n)), 0.0)
    out, done = [], 0
    for k in checkpoints:
        s.step(k - done)
        done = k
        out.append(s.get_fields())
    s.close()
    return out


@pytest.mark.parametrize("name,steps", [("blob64", 100), ("shell128", 200)])
def test_configured_lengths_fp32_against_fp64(Solver, name, steps):
    """The 64^3 and 128^3 workloads over their configured lengths (100 and
    200 steps from a zero state, the dipole driving the fields): the float32
    mode against the float64 path (itself equal to the oracle to 1e-12 per
    step at these sizes).  Bound per component: 1e-5 of the largest norm its
    field (E or H) reaches during the run (checked every quarter of the run),
    element-wise 5e-5 of the field's largest value.  At the end of the 128^3 run H
    has fallen to a ninth of its peak (the pulse is over) and H1, the
    component the x-directed dipole drives least, to 3 % of it: relative to
    their own final norms the H components then differ by 4e-5 to 1.5e-4
    (E: 4e-6), which is printed and bounded at 5e-4."""
    cps = [steps // 4, steps // 2, 3 * steps // 4, steps]
    r32 = _run_gpu_workload(Solver, name, "fp32_refine", cps)
    r64 = _run_gpu_workload(Solver, name, "fp64", cps)
    peak = [max(np.linalg.norm(g[f * 3:(f + 1) * 3].reshape(3, -1), axis=1).max()
                for g, _ in r64) for f in range(2)]
    peak_abs = [max(np.abs(g[f * 3:(f + 1) * 3]).max() for g, _ in r64) for f in range(2)]
    for (g32, t32), (g64, t64), k in zip(r32, r64, cps):
        assert t32 == pytest.approx(t64, rel=1e-12)
        err = [np.linalg.norm(g32[c] - g64[c]) for c in range(6)]
        own = [e / max(np.linalg.norm(g64[c]), 1e-300) for c, e in enumerate(err)]
        to_peak = [e / peak[c // 3] for c, e in enumerate(err)]
        emax = [np.abs(g32[c] - g64[c]).max() / peak_abs[c // 3] for c in range(6)]
        print(name, k, "fp32 vs fp64: relative to the field's peak", to_peak,
              "to the component's own norm", own, "max-abs to the field's peak", emax)
        assert max(to_peak) <= TOL32, (k, to_peak)
        assert max(own) <= 5e-4, (k, own)
        assert max(emax) <= MAXABS_FACTOR32 * TOL32, (k, emax)


def test_mms16_fp32_refine(Solver):
    w = workloads.make("mms16")
    prob = maxwell.Problem(w.N, w.p, 1.0, 1.0, 0.0, w.dt)
    quad = mms.Quadrature(w.N, w.p)
    E, H = mms.mms_initial(prob, quad)
    s = Solver(w.N, w.p, "fp32_refine")
    s.set_material(w.material.eps_r, w.material.mu_r, w.material.sigma_nd)
    s.factor(w.dt)
    s.set_fields(np.stack(E + H), 0.0)
    s.step(w.steps)
    E, H, t = prob.run(E, H, 0.0, w.steps)
    got, _ = s.get_fields()
    # H starts at zero; compare each field against the norm of its own
    # reference, the H part after 10 small steps is ~1e-2 of E
    compare_state(got, E, H, TOL32, "mms16 fp32")


def test_repeatable_bitwise(Solver):
    """No atomics on the hot path: the same steps give identical bits."""
    N, p = 6, 2
    eps, mu, sig, src = random_setup(N, p, seed=3)
    prob = maxwell.Problem(N, p, eps, mu, sig, 0.05, src)
    E, H = constrained_random_state(prob, 1)
    outs = []
    for _ in range(2):
        s = make_gpu(Solver, N, p, eps, mu, sig, 0.05, src)
        s.set_fields(np.stack(E + H), 0.0)
        s.step(5)
        outs.append(s.get_fields()[0])
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_profiling_pass_equals_graph_steps(Solver, precision):
    """The eager profiling pass (the per-kernel timings of bench.py) runs the
    same kernels as the captured graph: the same state after the same steps,
    bit for bit, that state equal to the oracle's, and one record per launch
    of a step."""
    N, p = 45, 3  # n = 48: partitioned shared-axis solves, mixed-axis rounds
    eps, mu, sig, src = random_setup(N, p, seed=11)
    dt = 0.5 / N
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    E, H = constrained_random_state(prob, 2)
    outs = []
    for mode in ("graph", "profile"):
        s = make_gpu(Solver, N, p, eps, mu, sig, dt, src, precision)
        s.set_fields(np.stack(E + H), 0.0)
        if mode == "graph":
            s.step(3)
        else:
            s.profile(3)
            launches = s.profile_read()
        outs.append(s.get_fields())
        s.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]
    E3, H3, _ = prob.run(E, H, 0.0, 3)
    compare_state(outs[1][0], E3, H3, TOL64 if precision == "fp64" else TOL32,
                  ("profiling pass", precision))
    kinds = [L["kind"] for L in launches]
    assert kinds.count("rhs_E") == 2 and kinds.count("rhs_H") == 2
    # the float32 mode adds the old state in the last solves of each stage
    nacc = sum(L["nacc"] for L in launches)
    assert nacc == (12 if precision == "fp32_refine" else 0)
    assert all(L["ms"] > 0 for L in launches)


def test_resume_equals_uninterrupted(Solver):
    N, p = 5, 2
    eps, mu, sig, src = random_setup(N, p, seed=4)
    prob = maxwell.Problem(N, p, eps, mu, sig, 0.05, src)
    E, H = constrained_random_state(prob, 2)
    s = make_gpu(Solver, N, p, eps, mu, sig, 0.05, src)
    s.set_fields(np.stack(E + H), 0.0)
    s.step(6)
    full, t_full = s.get_fields()
    s.set_fields(np.stack(E + H), 0.0)
    s.step(3)
    mid, t_mid = s.get_fields()
    s.set_fields(mid, t_mid)
    s.step(3)
    resumed, t_res = s.get_fields()
    assert np.array_equal(full, resumed) and t_full == t_res


@pytest.mark.parametrize("N,p,V", [(5, 2, 7), (12, 3, 20), (50, 2, 64)])
def test_bspline_averaged_material_steps(Solver, N, p, V):
    """B-spline-weighted material map: steps on the GPU against the oracle
    stepping with the oracle's own averaged material."""
    mat = workloads.blob_map(V, 40 + N)
    src = workloads.DipoleSource(xs=(0.4, 0.55, 0.5), f0=2.0, t0=0.05, width=0.3)
    dt = 0.5 / N
    prob = maxwell.problem_from_voxels(N, p, mat, dt, src, mapping="bspline_avg")
    s = Solver(N, p, "fp64")
    s.set_material(mat.eps_r, mat.mu_r, mat.sigma_nd, mapping="bspline_avg")
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.factor(dt)
    E, H = constrained_random_state(prob, 5)
    s.set_fields(np.stack(E + H), 0.02)
    s.step(2)
    E, H, _ = prob.run(E, H, 0.02, 2)
    got, _ = s.get_fields()
    compare_state(got, E, H, TOL64, ("bspline_avg", N, p, V))


@pytest.mark.parametrize("N,p", [(4, 2), (9, 3), (50, 2)])
def test_local_time_step_steps(Solver, N, p):
    """Per-test-function local time step: GPU steps against the oracle."""
    eps, mu, sig, src = random_setup(N, p, seed=300 + N)
    n = N + p
    dt = 0.5 / N
    tau = np.random.default_rng(N).uniform(0.2 * dt, 1.5 * dt, (n, n, n))
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src, local_dt=tau)
    s = Solver(N, p, "fp64")
    s.set_material_dof(eps, mu, sig)
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.set_local_dt(tau)
    s.factor(dt)
    E, H = constrained_random_state(prob, 6)
    s.set_fields(np.stack(E + H), 0.01)
    s.step(2)
    E, H, t = prob.run(E, H, 0.01, 2)
    got, tg = s.get_fields()
    assert tg == pytest.approx(t, rel=1e-14)
    compare_state(got, E, H, TOL64, ("local dt", N, p))


@pytest.mark.parametrize("precision,tol,res64", [("fp64", TOL64, None),
                                                 ("fp32_refine", TOL32, None),
                                                 ("fp32_refine", TOL32, 0),
                                                 ("fp32_refine", TOL32, 15)])
def test_shell32_subrun_50_steps(Solver, precision, tol, res64):
    """The 32^3 p=2 sub-run of the 256^3 shell workload (same voxel map):
    all 50 steps of its dt against the float64 oracle, per component (and
    per field, printed); the float32 mode with its default residual
    arithmetic, all-float32 (0) and all-float64 (15) increments."""
    got, E, H = _workload_pair(Solver, "shell32", 50, precision, res64)
    fields = {"E": rel_l2(got[:3], np.stack(E)), "H": rel_l2(got[3:], np.stack(H))}
    comp = compare_state(got, E, H, tol, ("shell32", precision, res64))
    print("shell32", precision, res64, "per-field relative L2:", fields, "per component:", comp)


def test_singular_pivot_reported_and_context_usable(Solver):
    """ADI_ESINGULAR: with the pivot floor raised above every pivot ratio of
    the pivot-free LU (|U_rr| / |A_rr| <= 1 for these matrices) adi_factor
    reports it; the context refuses to step and stays usable: with the
    default floor it factors and steps as before.  (The shared mass factors
    are checked first; adding alpha S with alpha >= 0 only raises the pivot
    ratios of the material-modified factors, so their check cannot trip
    before the shared one.)"""
    from paper_2103_06998_amd import _lib
    N, p = 6, 3
    eps, mu, sig, src = random_setup(N, p, seed=31)
    dt = 0.3
    prob = maxwell.Problem(N, p, eps, mu, sig, dt, src)
    s = make_gpu(Solver, N, p, eps, mu, sig, dt, src)
    s.set_pivot_floor(2.0)
    with pytest.raises(_lib.AdiError) as ei:
        s.factor(dt)
    assert ei.value.status == _lib.ADI_ESINGULAR
    assert b"pivot" in s.lib.adi_last_error(s.h)
    with pytest.raises(_lib.AdiError) as ei:
        s.step(1)
    assert ei.value.status == _lib.ADI_ESTATE
    s.set_pivot_floor(1e-14)
    s.factor(dt)
    E, H = constrained_random_state(prob, 3)
    s.set_fields(np.stack(E + H), 0.0)
    s.step(2)
    E, H, _ = prob.run(E, H, 0.0, 2)
    compare_state(s.get_fields()[0], E, H, TOL64, "after ESINGULAR")

"""Patches with a different element count per axis (the paper reorders each
right-hand side into N_x rows of N_y N_z columns, so N_x, N_y and N_z are
independent): the HIP path through the C ABI against the float64 oracle,
which builds each axis's 1D matrices from its own knot vector."""
import numpy as np
import pytest

import workloads
from oracle import maxwell, mms

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5


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


def shape_of(Ns, p):
    return (Ns[2] + p, Ns[1] + p, Ns[0] + p)


def random_problem(Ns, p, seed, dt):
    shape = shape_of(Ns, p)
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1.0, 50.0, shape)
    mu = rng.uniform(0.5, 2.0, shape)
    sig = rng.uniform(0.0, 20.0, shape)
    src = workloads.DipoleSource(xs=tuple(rng.uniform(0.1, 0.9, 3)), comp=seed % 3, amp=1.3,
                                 f0=2.0, t0=0.05, width=0.3)
    prob = maxwell.Problem(Ns, p, eps, mu, sig, dt, src)
    F = rng.standard_normal((6,) + shape)
    E, H = prob.constrain(list(F[:3]), list(F[3:]))
    return prob, E, H


def gpu_solver(Solver, prob, precision):
    s = Solver(prob.Ns, prob.p, precision)
    s.set_material_dof(prob.eps, prob.mu, prob.sig)
    src = prob.source
    s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
    s.factor(prob.dt)
    return s


def max_abs_rel(a, b):
    """Largest element-wise difference over the largest reference value (a
    component that is zero everywhere, e.g. E1 with a single y element at
    p = 1, must come out exactly zero)."""
    m = np.abs(b).max()
    return np.abs(a - b).max() / (m if m > 0 else 1.0)


def check(got, ref, tol, label):
    errs = [rel_l2(got[c], ref[c]) for c in range(len(ref))]
    emax = [max_abs_rel(got[c], ref[c]) for c in range(len(ref))]
    factor = 1.0 if tol <= TOL64 else 5.0
    assert max(errs) <= tol and max(emax) <= factor * tol, (label, errs, emax)
    return errs


# (12, 20, 33) p=3: all lines short (one lane per line); (45, 20, 60) p=3:
# x and z lines long enough for the partitioned solve, y lines not, so
# rounds mix descriptors of different lengths; (60, 7, 2) p=2: flat.
CASES = [((12, 20, 33), 3), ((45, 20, 60), 3), ((60, 7, 2), 2), ((3, 1, 5), 1)]


@pytest.mark.parametrize("Ns,p", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_full_steps_non_cubic(Solver, Ns, p, precision):
    prob, E, H = random_problem(Ns, p, seed=sum(Ns) + p, dt=0.5 / max(Ns))
    s = gpu_solver(Solver, prob, precision)
    assert s.shape == prob.shape
    s.set_fields(np.stack(E + H), 0.01)
    s.step(2)
    E, H, t = prob.run(E, H, 0.01, 2)
    got, tg = s.get_fields()
    assert tg == pytest.approx(t, rel=1e-14)
    errs = check(got, E + H, TOL64 if precision == "fp64" else TOL32, (Ns, p, precision))
    print("non-cubic", Ns, p, precision, errs)


@pytest.mark.parametrize("Ns,p", CASES[:2])
@pytest.mark.parametrize("stage,sub", [(0, 1), (0, 2), (1, 1), (1, 2)])
def test_stages_non_cubic(Solver, Ns, p, stage, sub):
    """Right-hand sides and 1D solves of one stage on their own."""
    prob, E, H = random_problem(Ns, p, seed=3, dt=0.07)
    s = gpu_solver(Solver, prob, "fp64")
    t = 0.2
    if stage == 0:
        fields = {"E1": E[0], "E2": E[1], "E3": E[2], "H1": H[0], "H2": H[1], "H3": H[2]}
        ref = [prob.rhs_E(sub, fields, c, prob.source_time(sub, t)) for c in range(3)]
        got = s.rhs(0, sub, np.stack(E + H), t)
    else:
        En = [1.7 * e + 0.3 for e in prob.constrain(E, H)[0]]
        En = prob.constrain(En, H)[0]
        fields = {"H1": H[0], "H2": H[1], "H3": H[2], "E1": E[0], "E2": E[1], "E3": E[2],
                  "E1'": En[0], "E2'": En[1], "E3'": En[2]}
        ref = [prob.rhs_H(sub, fields, c) for c in range(3)]
        got = s.rhs(1, sub, np.stack(H + E + En), t)
    check(got, ref, TOL64, ("rhs", Ns, stage, sub))
    kind = "E" if stage == 0 else "H"
    R = [maxwell.zero_boundary(r, maxwell.dirichlet_axes(kind, c)) for c, r in enumerate(ref)]
    sol = [prob.solve3(R[c], kind, c, maxwell.MOD_AXIS[sub][c] if kind == "E" else None)
           for c in range(3)]
    check(s.solve(stage, sub, np.stack(R)), sol, TOL64, ("solve", Ns, stage, sub))


@pytest.mark.parametrize("Ns,p", [((6, 9, 4), 2), ((5, 3, 8), 3)])
def test_mms_projection_and_errors_non_cubic(Solver, Ns, p):
    """Projection of the manufactured solution and its error norms on a
    patch of Nx x Ny x Nz elements, against the oracle (same tolerance
    reasoning as the cubic test)."""
    prob = maxwell.Problem(Ns, p, 1.0, 1.0, 0.0, 0.01)
    quad = mms.Quadrature(Ns, p)
    t = 0.3
    E, H = mms.mms_initial(prob, quad, t)
    s = Solver(Ns, p, "fp64")
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(0.01)
    s.mms_project(t=t)
    got, _ = s.get_fields()
    check(got, list(E) + list(H), 1e-10, ("mms projection", Ns, p))
    ref = mms.errors(quad, [got[0], got[1], got[2]], [got[3], got[4], got[5]], t)
    err = s.mms_errors()
    for k in ref:
        assert err[k] == pytest.approx(ref[k], rel=1e-10), k
    assert s.mms_errors_noalloc() == err


def test_voxel_material_non_cubic(Solver):
    """Greville and B-spline-averaged voxel maps on a non-cubic patch."""
    Ns, p = (10, 6, 14), 2
    mat = workloads.blob_map(24, 5)
    src = workloads.DipoleSource(xs=(0.4, 0.55, 0.5), f0=2.0, t0=0.05, width=0.3)
    for mapping in ("greville", "bspline_avg"):
        prob = maxwell.problem_from_voxels(Ns, p, mat, 0.04, src, mapping=mapping)
        s = Solver(Ns, p, "fp64")
        s.set_material(mat.eps_r, mat.mu_r, mat.sigma_nd, mapping=mapping)
        s.set_source(src.xs, src.comp, src.amp, src.f0, src.t0, src.width)
        s.factor(0.04)
        F = np.random.default_rng(2).standard_normal((6,) + prob.shape)
        E, H = prob.constrain(list(F[:3]), list(F[3:]))
        s.set_fields(np.stack(E + H), 0.0)
        s.step(2)
        E, H, _ = prob.run(E, H, 0.0, 2)
        check(s.get_fields()[0], E + H, TOL64, mapping)


def test_closure_needs_cubic_patch(Solver):
    from paper_2103_06998_amd import _lib
    s = Solver((4, 5, 6), 2, "fp64")
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(0.05)
    with pytest.raises(_lib.AdiError) as ei:
        s.closure_mark()
    assert ei.value.status == _lib.ADI_EINVAL

"""Manufactured solution on the GPU: projection and error norms against the
float64 oracle, and the paper's convergence results (section "Numerical code
verification with manufactured solution", Figs. 2-4) reproduced on the GPU."""
import json
import os

import numpy as np
import pytest

from oracle import maxwell, mms

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "mms_bounds.json")


@pytest.fixture(scope="module")
def Solver():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_06998_amd.solver import Solver as S
    return S


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("N,p,t", [(16, 2, 0.0), (5, 3, 0.3), (50, 2, 0.7)])
def test_projection_matches_oracle(Solver, N, p, t):
    """Tolerance 1e-10: the right-hand sides are sums of ~(p+1)^3 q^3 products
    of sines (a few ulp apart between the GPU and numpy), and the 3D mass
    solve amplifies their relative error by up to cond(M)^3 (~1e3 at p = 2,
    ~2e4 at p = 3)."""
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, 0.01)
    quad = mms.Quadrature(N, p)
    E, H = mms.mms_initial(prob, quad, t)
    s = Solver(N, p, "fp64")
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(0.01)
    s.mms_project(t=t)
    got, tg = s.get_fields()
    assert tg == t
    ref = np.stack(list(E) + list(H))
    for c in range(6):
        if np.linalg.norm(ref[c]) > 0:
            assert rel_l2(got[c], ref[c]) <= 1e-10, c
        else:
            assert np.max(np.abs(got[c])) <= 1e-14


@pytest.mark.parametrize("N,p,steps", [(16, 2, 0), (16, 2, 10), (6, 3, 7)])
def test_error_norms_match_oracle(Solver, N, p, steps):
    dt = 0.02
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, dt)
    quad = mms.Quadrature(N, p)
    s = Solver(N, p, "fp64")
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(dt)
    s.mms_project(t=0.0)
    s.step(steps)
    got = s.mms_errors()
    F, t = s.get_fields()
    ref = mms.errors(quad, list(F[:3]), list(F[3:]), t)
    for k in ("E_L2", "E_Hcurl", "H_L2", "H_Hcurl"):
        assert got[k] == pytest.approx(ref[k], rel=1e-10, abs=1e-14), k


def test_paper_error_bounds_and_second_order(Solver):
    """Max over t in [0, 1] of the L2 and H(curl) errors at 16^3 p=2 for
    tau = 1/10 and 1/1280 within the bounds the paper prints, and second
    order in tau."""
    from paper_2103_06998_amd import mms_study
    g = json.load(open(GOLDEN))
    r10 = mms_study.run_tau(16, 2, 10)
    r1280 = mms_study.run_tau(16, 2, 1280)
    for f in ("E", "H"):
        assert r10[f + "_L2"] < g["L2_error_bound"]["10"]
        assert r1280[f + "_L2"] < g["L2_error_bound"]["1280"]
        assert r10[f + "_Hcurl"] < g["Hcurl_error_bound"]["10"]
        assert r1280[f + "_Hcurl"] < g["Hcurl_error_bound"]["1280"]
    r20, r40 = mms_study.run_tau(16, 2, 20), mms_study.run_tau(16, 2, 40)
    for f in ("E_L2", "H_L2"):
        order = np.log2(r20[f] / r40[f])
        assert order > 1.8, (f, order)


def _field_values(quad, seed):
    """Six smooth, non-polynomial fields at the quadrature points (not a
    Maxwell solution: the projection takes any data)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in range(6):
        a, b, d = rng.uniform(0.5, 3.0, 3)
        ph = rng.uniform(0, np.pi, 3)
        out.append(np.cos(a * quad.X + ph[0]) * np.sin(b * quad.Y + ph[1]) *
                   np.exp(-d * (quad.Z - 0.4) ** 2) + 0.1 * c)
    return out


@pytest.mark.parametrize("N,p,q", [(6, 2, 5), (9, 3, 4), (4, 1, 7), (50, 2, 3)])
def test_general_projection_matches_oracle(Solver, N, p, q):
    """adi_project of caller-given values at the Gauss points against the
    oracle's L2 projection (same tolerance reasoning as above)."""
    prob = maxwell.Problem(N, p, 1.0, 1.0, 0.0, 0.01)
    quad = mms.Quadrature(N, p, q)
    vals = _field_values(quad, N + 10 * p)
    E, H = mms.project(prob, quad, vals)
    s = Solver(N, p, "fp64")
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(0.01)
    s.project(np.stack(vals), q, t=0.25)
    got, tg = s.get_fields()
    assert tg == 0.25
    ref = np.stack(list(E) + list(H))
    for c in range(6):
        assert rel_l2(got[c], ref[c]) <= 1e-10, (c, rel_l2(got[c], ref[c]))


def test_general_projection_rejects_nonfinite(Solver):
    from paper_2103_06998_amd import _lib
    N, p, q = 3, 2, 3
    s = Solver(N, p, "fp64")
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(0.01)
    vals = np.zeros((6, N * q, N * q, N * q))
    vals[2, 1, 1, 1] = np.nan
    with pytest.raises(_lib.AdiError) as ei:
        s.project(vals, q)
    assert ei.value.status == _lib.ADI_ENONFINITE

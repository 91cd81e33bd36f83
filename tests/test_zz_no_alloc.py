"""The allocation-free error entry point (adi_mms_errors_noalloc) against the
allocating one (adi_mms_errors): two calls in a row through the C ABI, the
second on a smaller grid, each bit for bit equal to the allocating entry
point's result on the same state (same kernel, same block order)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Solver():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_06998_amd.solver import Solver as S
    return S


def _state(Solver, N, p, precision, steps):
    s = Solver(N, p, precision)
    s.set_material_dof(1.0, 1.0, 0.0)
    s.factor(0.02)
    s.mms_project(t=0.1)
    s.step(steps)
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_noalloc_errors_equal_allocating_errors(Solver, precision):
    big = _state(Solver, 20, 3, precision, 3)
    small = _state(Solver, 7, 2, precision, 2)
    q_big, q_small = 6, 4
    got_big = big.mms_errors_noalloc(q_big)
    got_small = small.mms_errors_noalloc(q_small)   # second call, smaller input
    ref_big = big.mms_errors(q_big)
    ref_small = small.mms_errors(q_small)
    for got, ref in ((got_big, ref_big), (got_small, ref_small)):
        for k in ref:
            assert np.isfinite(ref[k]) and ref[k] > 0, (k, ref)
            assert got[k] == ref[k], (k, got[k], ref[k])
    # a repeat on the larger grid after the smaller one (the array keeps the
    # last call's contents) gives the same numbers again
    assert big.mms_errors_noalloc(q_big) == ref_big

"""The C-ABI library loads on a machine without a GPU, exports every symbol
declared in include/adimx.h, and rejects invalid input on the host before any
device work (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2103_06998_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2103_06998_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "adimx.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(adi_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("adi_create", "adi_set_material", "adi_factor", "adi_step",
                     "adi_get_fields", "adi_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def _ctx(lib, N=3, p=2, prec=0):
    h = ctypes.c_void_p()
    st = lib.adi_create(ctypes.byref(h), N, N, N, p, prec, None)
    return st, h


def test_host_validation_errors(lib):
    h = ctypes.c_void_p()
    assert lib.adi_create(ctypes.byref(h), 0, 0, 0, 2, 0, None) == _lib.ADI_EINVAL
    assert lib.adi_create(ctypes.byref(h), 4, 4, 4, 0, 0, None) == _lib.ADI_EINVAL
    assert lib.adi_create(ctypes.byref(h), 4, 4, 4, 5, 0, None) == _lib.ADI_EINVAL
    assert lib.adi_create(ctypes.byref(h), 4, 0, 4, 2, 0, None) == _lib.ADI_EINVAL
    # (nx+p)(ny+p)(nz+p) coefficients per component must stay below 2^31
    assert lib.adi_create(ctypes.byref(h), 1290, 1290, 1290, 1, 0, None) == _lib.ADI_EINVAL
    # element counts may differ per axis
    assert lib.adi_create(ctypes.byref(h), 4, 5, 6, 2, 0, None) == _lib.ADI_OK
    dims = (ctypes.c_int * 3)()
    assert lib.adi_dims(h, dims) == _lib.ADI_OK and list(dims) == [6, 7, 8]
    assert lib.adi_ncoef(h) == 6
    assert lib.adi_workspace_bytes(h) > 6 * 6 * 7 * 8 * 8
    lib.adi_destroy(h)
    assert lib.adi_create(ctypes.byref(h), 4, 4, 4, 2, 7, None) == _lib.ADI_EINVAL
    st, h = _ctx(lib)
    assert st == _lib.ADI_OK
    try:
        n = lib.adi_ncoef(h)
        assert n == 5
        assert lib.adi_workspace_bytes(h) > 6 * n ** 3 * 8
        D = n ** 3
        one = np.ones(D)
        bad = np.ones(D)
        bad[7] = 0.0
        neg = np.zeros(D)
        neg[3] = -1.0
        nan = np.ones(D)
        nan[1] = np.nan
        d = _lib.dptr
        assert lib.adi_set_material_dof(h, d(bad), d(one), d(np.zeros(D))) == _lib.ADI_EINVAL
        assert b"eps" in lib.adi_last_error(h)
        assert lib.adi_set_material_dof(h, d(one), d(bad), d(np.zeros(D))) == _lib.ADI_EINVAL
        assert lib.adi_set_material_dof(h, d(one), d(one), d(neg)) == _lib.ADI_EINVAL
        assert lib.adi_set_material_dof(h, d(nan), d(one), d(np.zeros(D))) == _lib.ADI_EINVAL
        v = np.ones(8)
        assert lib.adi_set_material(h, d(v), d(v), d(v), 2, 2, 2, 9) == _lib.ADI_EINVAL
        vb = v.copy()
        vb[0] = -2
        assert lib.adi_set_material(h, d(vb), d(v), d(v), 2, 2, 2, 0) == _lib.ADI_EINVAL
        # factor before material, step before factor
        assert lib.adi_factor(h, 0.1) == _lib.ADI_ESTATE
        assert lib.adi_step(h, 1) == _lib.ADI_ESTATE
        assert lib.adi_step(h, -1) == _lib.ADI_EINVAL
        xs = np.array([0.5, 0.5, 1.5])
        assert lib.adi_set_source(h, d(xs), 0, 1.0, 2.0, 0.5, 0.2) == _lib.ADI_EINVAL
        xs = np.array([0.5, 0.5, 0.5])
        assert lib.adi_set_source(h, d(xs), 3, 1.0, 2.0, 0.5, 0.2) == _lib.ADI_EINVAL
        assert lib.adi_set_source(h, d(xs), 0, 1.0, 2.0, 0.5, 0.0) == _lib.ADI_EINVAL
        f = np.zeros(6 * D)
        f[5] = np.inf
        assert lib.adi_set_fields(h, d(f), 0.0) == _lib.ADI_ENONFINITE
        assert lib.adi_set_material_dof(h, d(one), d(one), d(np.zeros(D))) == _lib.ADI_OK
        assert lib.adi_factor(h, float("nan")) == _lib.ADI_EINVAL
        assert lib.adi_factor(h, -1.0) == _lib.ADI_EINVAL
        assert lib.adi_set_pivot_floor(h, -1.0) == _lib.ADI_EINVAL
        assert lib.adi_set_pivot_floor(h, float("inf")) == _lib.ADI_EINVAL
        assert lib.adi_set_pivot_floor(h, 0.5) == _lib.ADI_OK
        assert lib.adi_set_residual64(h, -1) == _lib.ADI_EINVAL
        assert lib.adi_set_residual64(h, 16) == _lib.ADI_EINVAL
        assert lib.adi_set_residual64(h, 15) == _lib.ADI_OK
    finally:
        lib.adi_destroy(h)


def test_network_host_validation(lib):
    h = ctypes.c_void_p()
    assert lib.adi_nn_create(ctypes.byref(h), 0, 32, 6, None) == _lib.ADI_EINVAL
    assert lib.adi_nn_create(ctypes.byref(h), 17, 32, 6, None) == _lib.ADI_EINVAL
    assert lib.adi_nn_create(ctypes.byref(h), 16, 16, 6, None) == _lib.ADI_EINVAL
    assert lib.adi_nn_create(ctypes.byref(h), 16, 32, 0, None) == _lib.ADI_EINVAL
    assert lib.adi_nn_create(None, 16, 32, 6, None) == _lib.ADI_EINVAL
    assert lib.adi_nn_param_count(None) == _lib.ADI_EINVAL
    assert lib.adi_copy_state(None, None) == _lib.ADI_EINVAL
    assert lib.adi_step_closure(None, None, 1, ctypes.c_float(0.0)) == _lib.ADI_EINVAL


def test_noalloc_errors_host_validation(lib):
    """adi_mms_errors_noalloc checks its sizes against the fixed 1 MiB device
    array on the host, before touching the device."""
    out = np.zeros(4)
    d = _lib.dptr
    st, h = _ctx(lib, N=700, p=4)
    assert st == _lib.ADI_OK
    try:
        # 700 * 16 * (2*4 + 4) + 8192 float64 values do not fit in 1 MiB
        assert lib.adi_mms_errors_noalloc(h, 16, d(out)) == _lib.ADI_ENOMEM
        assert b"scratch" in lib.adi_last_error(h)
        assert lib.adi_mms_errors_noalloc(h, 0, d(out)) == _lib.ADI_EINVAL
        assert lib.adi_mms_errors_noalloc(h, 17, d(out)) == _lib.ADI_EINVAL
        # fits (700 * 1 * 12 + 8192), but no state yet
        assert lib.adi_mms_errors_noalloc(h, 1, d(out)) == _lib.ADI_ESTATE
        assert lib.adi_mms_errors_noalloc(h, 1, None) == _lib.ADI_EINVAL
    finally:
        lib.adi_destroy(h)
    assert lib.adi_mms_errors_noalloc(None, 3, d(out)) == _lib.ADI_EINVAL


def test_project_host_validation(lib):
    st, h = _ctx(lib)
    try:
        vals = np.zeros(6 * 9 ** 3)
        assert lib.adi_project(h, _lib.dptr(vals), 3, 0.0) == _lib.ADI_ESTATE
        assert lib.adi_project(h, None, 3, 0.0) == _lib.ADI_EINVAL
        assert lib.adi_project(h, _lib.dptr(vals), 3, float("inf")) == _lib.ADI_EINVAL
    finally:
        lib.adi_destroy(h)

"""ctypes declarations of the libadimx C ABI (include/adimx.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadimx.so")

ADI_OK, ADI_EINVAL, ADI_ENOMEM, ADI_EHIP, ADI_ESINGULAR, ADI_ENONFINITE, ADI_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
ADI_FP64, ADI_FP32_REFINE = 0, 1
ADI_MAP_GREVILLE, ADI_MAP_BSPLINE_AVG = 0, 1
ADI_RES64_E1, ADI_RES64_H1, ADI_RES64_E2, ADI_RES64_H2 = 1, 2, 4, 8
ADI_RES64_DEFAULT = ADI_RES64_E2

STATUS_NAMES = {0: "ADI_OK", -1: "ADI_EINVAL", -2: "ADI_ENOMEM", -3: "ADI_EHIP",
                -4: "ADI_ESINGULAR", -5: "ADI_ENONFINITE", -6: "ADI_ESTATE"}

# Every exported symbol and its (restype, argtypes).
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_F = ctypes.POINTER(ctypes.c_float)
SIGNATURES = {
    "adi_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _I, _I, _P]),
    "adi_ncoef": (_I, [_P]),
    "adi_dims": (_I, [_P, ctypes.POINTER(_I)]),
    "adi_workspace_bytes": (ctypes.c_size_t, [_P]),
    "adi_bind_workspace": (_I, [_P, _P, ctypes.c_size_t]),
    "adi_set_material": (_I, [_P, _D, _D, _D, _I, _I, _I, _I]),
    "adi_set_material_dof": (_I, [_P, _D, _D, _D]),
    "adi_factor": (_I, [_P, ctypes.c_double]),
    "adi_set_pivot_floor": (_I, [_P, ctypes.c_double]),
    "adi_set_residual64": (_I, [_P, _I]),
    "adi_set_local_dt": (_I, [_P, _D]),
    "adi_set_source": (_I, [_P, _D, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double]),
    "adi_set_fields": (_I, [_P, _D, ctypes.c_double]),
    "adi_step": (_I, [_P, _I]),
    "adi_get_fields": (_I, [_P, _D, _D]),
    "adi_fields_device": (_I, [_P, ctypes.POINTER(_P), ctypes.POINTER(_I)]),
    "adi_sync": (_I, [_P]),
    "adi_last_error": (ctypes.c_char_p, [_P]),
    "adi_destroy": (None, [_P]),
    "adi_rhs": (_I, [_P, _I, _I, _D, ctypes.c_double, _D]),
    "adi_solve": (_I, [_P, _I, _I, _D]),
    "adi_mms_project": (_I, [_P, _I, ctypes.c_double]),
    "adi_mms_errors": (_I, [_P, _I, _D]),
    "adi_project": (_I, [_P, _D, _I, ctypes.c_double]),
    "adi_mms_errors_noalloc": (_I, [_P, _I, _D]),
    "adi_profile_run": (_I, [_P, _I]),
    "adi_profile_read": (_I, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                              ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                              ctypes.POINTER(ctypes.c_float)]),
    # learned closure
    "adi_nn_create": (_I, [ctypes.POINTER(_P), _I, _I, _I, _P]),
    "adi_nn_param_count": (_I, [_P]),
    "adi_nn_set_params": (_I, [_P, _F]),
    "adi_nn_get_params": (_I, [_P, _F]),
    "adi_nn_forward": (_I, [_P, _P, _P, _I, _I, _I]),
    "adi_nn_backward": (_I, [_P, _P]),
    "adi_nn_get_grads": (_I, [_P, _F]),
    "adi_nn_adam": (_I, [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _I]),
    "adi_nn_mse": (_I, [_P, _P, _P, ctypes.c_size_t, _P, _D]),
    "adi_nn_last_error": (ctypes.c_char_p, [_P]),
    "adi_nn_destroy": (None, [_P]),
    "adi_copy_state": (_I, [_P, _P]),
    "adi_closure_mark": (_I, [_P]),
    "adi_closure_features": (_I, [_P, _P, _P]),
    "adi_closure_target": (_I, [_P, _P, _P, _P]),
    "adi_closure_apply": (_I, [_P, _P, _P]),
    "adi_step_closure": (_I, [_P, _P, _I, ctypes.c_float]),
    "adi_closure_rejected": (_I, [_P, ctypes.POINTER(_I)]),
}

_lib = None


class AdiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libadimx.so (cached).  Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2103_06998_amd.build` (there is no fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def dptr(a):
    """ctypes double* of a C-contiguous float64 numpy array."""
    return a.ctypes.data_as(_D)

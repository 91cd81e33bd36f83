"""Object API over the libadimx C ABI.

PyTorch is used only for device memory (the workspace tensor the library
carves its buffers from) and for the HIP stream the library enqueues on.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

PRECISIONS = {"fp64": _lib.ADI_FP64, "fp32_refine": _lib.ADI_FP32_REFINE}


class Solver:
    """ADI time stepper for a patch of degree-p B-splines.

    Parameters
    ----------
    N : elements per axis (an int for a cube, or (Nx, Ny, Nz)).
    p : B-spline degree (1 <= p <= 4).
    precision : "fp64" or "fp32_refine".
    device : torch device string; its current stream is used.
    """

    def __init__(self, N: int, p: int, precision: str = "fp64", device: str = "cuda:0",
                 stream=None):
        import torch

        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the ADI step runs only in the HIP library")
        self.p = int(p)
        self.Ns = tuple(int(v) for v in np.broadcast_to(np.asarray(N), (3,)))
        self.dims = tuple(v + self.p for v in self.Ns)          # (nx, ny, nz)
        self.shape = (self.dims[2], self.dims[1], self.dims[0])  # arrays: [z][y][x]
        self.D = int(np.prod(self.dims))
        if len(set(self.Ns)) == 1:  # a cube: one element count for every axis
            self.N, self.n = self.Ns[0], self.dims[0]
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        st = self.lib.adi_create(ctypes.byref(h), *self.Ns, self.p,
                                 PRECISIONS[precision], ctypes.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise _lib.AdiError(st, "adi_create")
        self.h = h
        nbytes = int(self.lib.adi_workspace_bytes(self.h))
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._check(self.lib.adi_bind_workspace(self.h, ctypes.c_void_p(self.workspace.data_ptr()),
                                                nbytes))

    # -- helpers -------------------------------------------------------------
    def _check(self, st: int):
        if st != 0:
            msg = self.lib.adi_last_error(self.h).decode()
            raise _lib.AdiError(st, msg)

    def _arr(self, a, count=None):
        a = np.ascontiguousarray(a, dtype=np.float64)
        if count is not None and a.size != count:
            raise ValueError(f"expected {count} values, got {a.size}")
        return a

    def close(self):
        if getattr(self, "h", None):
            self.lib.adi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ---------------------------------------------------------------
    MAPS = {"greville": _lib.ADI_MAP_GREVILLE, "bspline_avg": _lib.ADI_MAP_BSPLINE_AVG}

    def set_material(self, eps_r, mu_r, sigma_nd, mapping: str = "greville"):
        """Voxel material map (arrays shaped (Vz, Vy, Vx)) attached to the test
        functions by Greville sampling or the B-spline-weighted average."""
        e, m, s = (self._arr(v) for v in (eps_r, mu_r, sigma_nd))
        Vz, Vy, Vx = np.shape(eps_r)
        self._check(self.lib.adi_set_material(self.h, _lib.dptr(e), _lib.dptr(m), _lib.dptr(s),
                                              Vx, Vy, Vz, self.MAPS[mapping]))

    def set_material_dof(self, eps, mu, sigma_nd):
        D = self.D
        e, m, s = (self._arr(np.broadcast_to(np.asarray(v, float), self.shape), D)
                   for v in (eps, mu, sigma_nd))
        self._check(self.lib.adi_set_material_dof(self.h, _lib.dptr(e), _lib.dptr(m), _lib.dptr(s)))

    def set_source(self, xs, comp=0, amp=1.0, f0=2.0, t0=0.5, width=0.2):
        x = self._arr(xs, 3)
        self._check(self.lib.adi_set_source(self.h, _lib.dptr(x), int(comp), float(amp),
                                            float(f0), float(t0), float(width)))

    def set_local_dt(self, tau=None):
        """Per-DOF local time step in the row coefficients (None: dt)."""
        if tau is None:
            self._check(self.lib.adi_set_local_dt(self.h, None))
            return
        a = self._arr(np.broadcast_to(np.asarray(tau, float), self.shape), self.D)
        self._check(self.lib.adi_set_local_dt(self.h, _lib.dptr(a)))

    def set_pivot_floor(self, floor: float):
        """Smallest accepted pivot / diagonal ratio of the LU (default 1e-14)."""
        self._check(self.lib.adi_set_pivot_floor(self.h, float(floor)))

    def set_residual64(self, mask: int):
        """Float32 mode: stages whose increment is formed in float64
        arithmetic (OR of _lib.ADI_RES64_*; default: the E stage of
        substep 2).  Takes effect at the next factor()."""
        self._check(self.lib.adi_set_residual64(self.h, int(mask)))

    def factor(self, dt: float):
        self._check(self.lib.adi_factor(self.h, float(dt)))

    # -- state ---------------------------------------------------------------
    def set_fields(self, EH, t: float = 0.0):
        a = self._arr(EH, 6 * self.D)
        self._check(self.lib.adi_set_fields(self.h, _lib.dptr(a), float(t)))

    def get_fields(self):
        out = np.empty((6,) + self.shape)
        t = ctypes.c_double()
        self._check(self.lib.adi_get_fields(self.h, _lib.dptr(out), ctypes.byref(t)))
        return out, t.value

    def step(self, nsteps: int = 1):
        self._check(self.lib.adi_step(self.h, int(nsteps)))

    def sync(self):
        self._check(self.lib.adi_sync(self.h))

    def fields_device(self):
        ptr = ctypes.c_void_p()
        dt = ctypes.c_int()
        self._check(self.lib.adi_fields_device(self.h, ctypes.byref(ptr), ctypes.byref(dt)))
        return ptr.value, ("float64" if dt.value == 0 else "float32")

    # -- per-kernel timing -----------------------------------------------------
    KINDS = ("rhs_E", "rhs_H", "unused", "sweep_x", "sweep_yz", "sweep_xyz", "apply_xyz")

    def profile(self, nsteps: int):
        """Run nsteps eager steps with HIP events around every launch."""
        self._check(self.lib.adi_profile_run(self.h, int(nsteps)))

    def profile_read(self):
        """Launches of one step with their mean durations: list of dicts."""
        cap = 256
        kind = (ctypes.c_int * cap)()
        nd = (ctypes.c_int * cap)()
        nm = (ctypes.c_int * cap)()
        na = (ctypes.c_int * cap)()
        ms = (ctypes.c_float * cap)()
        nout = ctypes.c_int()
        self._check(self.lib.adi_profile_read(self.h, cap, ctypes.byref(nout), kind, nd, nm, na,
                                              ms))
        return [dict(kind=self.KINDS[kind[i]], ncomp=nd[i], nmod=nm[i], nacc=na[i],
                     ms=float(ms[i])) for i in range(min(cap, nout.value))]

    # -- single stages (testing) ---------------------------------------------
    def rhs(self, stage: int, sub: int, fields, t: float = 0.0):
        nf = 6 if stage == 0 else 9
        a = self._arr(fields, nf * self.D)
        out = np.empty((3,) + self.shape)
        self._check(self.lib.adi_rhs(self.h, int(stage), int(sub), _lib.dptr(a), float(t),
                                     _lib.dptr(out)))
        return out

    def solve(self, stage: int, sub: int, rhs):
        a = self._arr(rhs, 3 * self.D).copy()
        self._check(self.lib.adi_solve(self.h, int(stage), int(sub), _lib.dptr(a)))
        return a.reshape((3,) + self.shape)

    # -- learned closure (solver side) ----------------------------------------
    def copy_state_from(self, other: "Solver"):
        """Device copy of other's state and time into this solver (same n)."""
        self._check(self.lib.adi_copy_state(self.h, other.h))

    def closure_mark(self):
        """Remember the current state as the state before a coarse step."""
        self._check(self.lib.adi_closure_mark(self.h))

    def closure_features(self, x, scale):
        """x: float32 device tensor [n^3, 15]; scale: float32 device tensor [1]."""
        self._check(self.lib.adi_closure_features(self.h, ctypes.c_void_p(x.data_ptr()),
                                                  ctypes.c_void_p(scale.data_ptr())))

    def closure_target(self, fine: "Solver", scale, t):
        """t[v][c] = (fine - self) / scale (float32 device tensors)."""
        self._check(self.lib.adi_closure_target(fine.h, self.h, ctypes.c_void_p(scale.data_ptr()),
                                                ctypes.c_void_p(t.data_ptr())))

    def closure_apply(self, y, scale):
        self._check(self.lib.adi_closure_apply(self.h, ctypes.c_void_p(y.data_ptr()),
                                               ctypes.c_void_p(scale.data_ptr())))

    def step_closure(self, net, nsteps: int = 1, gate: float = 0.0):
        """nsteps coarse steps, each followed by the network's correction."""
        self._check(self.lib.adi_step_closure(self.h, net.h, int(nsteps), float(gate)))

    def closure_rejected(self) -> int:
        c = ctypes.c_int()
        self._check(self.lib.adi_closure_rejected(self.h, ctypes.byref(c)))
        return c.value

    # -- manufactured solution ------------------------------------------------
    def mms_project(self, q: int = 0, t: float = 0.0):
        """State = L2 projection of the manufactured solution at time t."""
        self._check(self.lib.adi_mms_project(self.h, int(q or self.p + 3), float(t)))

    def project(self, vals_qp, q: int, t: float = 0.0):
        """State = L2 projection of six component fields given at the Gauss
        points (array (6, Nz q, Ny q, Nx q), x fastest), time t."""
        a = self._arr(vals_qp, 6 * int(np.prod([Na * int(q) for Na in self.Ns])))
        self._check(self.lib.adi_project(self.h, _lib.dptr(a), int(q), float(t)))

    def mms_errors_noalloc(self, q: int = 0) -> dict:
        """mms_errors through the entry point that allocates no device memory."""
        out = np.empty(4)
        self._check(self.lib.adi_mms_errors_noalloc(self.h, int(q or self.p + 3), _lib.dptr(out)))
        return {"E_L2": out[0], "E_Hcurl": out[1], "H_L2": out[2], "H_Hcurl": out[3]}

    def mms_errors(self, q: int = 0) -> dict:
        """Absolute L2 and H(curl) errors of E and H against the manufactured
        solution at the current time."""
        out = np.empty(4)
        self._check(self.lib.adi_mms_errors(self.h, int(q or self.p + 3), _lib.dptr(out)))
        return {"E_L2": out[0], "E_Hcurl": out[1], "H_L2": out[2], "H_Hcurl": out[3]}

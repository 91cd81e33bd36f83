"""Learned closure of the coarse ADI step: network handle, training-pair
generation, training and evaluation.

Orchestration and argument marshalling only: the ADI steps, the network's
features, forward and backward passes, the loss and the Adam update all run
in libadimx's HIP kernels; PyTorch provides device buffers and the stream.

The closure replaces ``ratio`` fine steps of size dt by one coarse step of
size ratio * dt followed by a learned correction y = net(features):
    C = coarse step of S,   C <- C + s * net(C/s, (C-S)/s, material, source)
with s the RMS of C.  The network is trained on pairs that the solver
generates itself: the target is (F - C) / s with F the fine solution from
the same starting state S.
"""
from __future__ import annotations

import ctypes
import dataclasses
import time
from typing import List, Optional, Sequence

import numpy as np

from . import _lib
from .solver import Solver

N_FEATURES = 16
N_OUTPUTS = 6
HIDDEN = 32
SHAPES = [(N_FEATURES, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, N_OUTPUTS)]


def init_params(seed: int, shapes: Sequence = SHAPES, last_gain: float = 0.1) -> np.ndarray:
    """Seeded He-normal initial parameters (float32), the last layer scaled
    down so that the untrained correction starts small; biases zero."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ci, co) in enumerate(shapes):
        W = rng.standard_normal((27, ci, co)) * np.sqrt(2.0 / (27 * ci))
        if li == len(shapes) - 1:
            W *= last_gain
        parts += [W.ravel(), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


class Network:
    """Handle of the library's 3-layer 3x3x3 convolutional network."""

    def __init__(self, cin: int = N_FEATURES, chid: int = HIDDEN, cout: int = N_OUTPUTS,
                 device: str = "cuda:0", stream=None):
        import torch

        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the closure network runs only in the HIP library")
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cin, self.chid, self.cout = cin, chid, cout
        h = ctypes.c_void_p()
        st = self.lib.adi_nn_create(ctypes.byref(h), cin, chid, cout,
                                    ctypes.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise _lib.AdiError(st, "adi_nn_create")
        self.h = h
        self.nparams = int(self.lib.adi_nn_param_count(self.h))
        self.step_count = 0

    def _check(self, st: int):
        if st != 0:
            raise _lib.AdiError(st, self.lib.adi_nn_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.adi_nn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- parameters ------------------------------------------------------------
    def set_params(self, params: np.ndarray):
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {a.size}")
        self._check(self.lib.adi_nn_set_params(self.h, a.ctypes.data_as(_lib._F)))
        self.step_count = 0

    def get_params(self) -> np.ndarray:
        a = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.adi_nn_get_params(self.h, a.ctypes.data_as(_lib._F)))
        return a

    def get_grads(self) -> np.ndarray:
        a = np.empty(self.nparams, dtype=np.float32)
        self._check(self.lib.adi_nn_get_grads(self.h, a.ctypes.data_as(_lib._F)))
        return a

    # -- compute ---------------------------------------------------------------
    def forward(self, x, grid, y=None):
        """x: float32 device tensor [nz*ny*nx, cin]; grid = (nz, ny, nx)."""
        import torch

        nz, ny, nx = grid
        if x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != nz * ny * nx * self.cin:
            raise ValueError("x must be a contiguous float32 tensor of grid x cin values")
        if y is None:
            y = torch.empty((nz * ny * nx, self.cout), dtype=torch.float32, device=x.device)
        self._check(self.lib.adi_nn_forward(self.h, ctypes.c_void_p(x.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()), nx, ny, nz))
        return y

    def backward(self, dy):
        self._check(self.lib.adi_nn_backward(self.h, ctypes.c_void_p(dy.data_ptr())))

    def mse(self, y, target, dy=None, want_loss: bool = True):
        import torch

        if dy is None:
            dy = torch.empty_like(y)
        loss = ctypes.c_double()
        self._check(self.lib.adi_nn_mse(self.h, ctypes.c_void_p(y.data_ptr()),
                                        ctypes.c_void_p(target.data_ptr()), y.numel(),
                                        ctypes.c_void_p(dy.data_ptr()),
                                        ctypes.byref(loss) if want_loss else None))
        return (loss.value if want_loss else None), dy

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step_count += 1
        self._check(self.lib.adi_nn_adam(self.h, float(lr), float(beta1), float(beta2),
                                         float(eps), self.step_count))


# ------------------------------------------------------------------ pairs
@dataclasses.dataclass
class PairSet:
    grid: tuple            # (n, n, n)
    x: list                # float32 device tensors [n^3, 16]
    t: list                # float32 device tensors [n^3, 6]


def _solver(N, p, material, source, dt, precision="fp64"):
    s = Solver(N, p, precision)
    s.set_material(material.eps_r, material.mu_r, material.sigma_nd)
    if source is not None:
        s.set_source(source.xs, source.comp, source.amp, source.f0, source.t0, source.width)
    s.factor(dt)
    return s


def generate_pairs(N: int, p: int, materials, sources, dt_coarse: float, fine_sub: int,
                   pairs_per_map: int, every: int, warmup: int,
                   pairs: Optional[PairSet] = None, rollout_net: Optional[Network] = None,
                   gate: float = 0.0) -> PairSet:
    """Training pairs from the solver itself, per (material, source).

    From each sampled state S one coarse step gives C and fine_sub fine steps
    (dt_coarse / fine_sub) give F; the pair is (features of C, S) ->
    (F - C) / s.  The states S come from a fine trajectory (sampled after
    `warmup` fine steps, then every `every` fine steps), or, with
    rollout_net, from a closure trajectory of that network (warmup and every
    counted in coarse steps): the states the closure itself visits."""
    import torch

    n = N + p
    D = n ** 3
    if pairs is None:
        pairs = PairSet((n, n, n), [], [])
    dt_fine = dt_coarse / fine_sub
    for mat, src in zip(materials, sources):
        if rollout_net is None:
            traj = _solver(N, p, mat, src, dt_fine)
            advance = traj.step
        else:
            traj = _solver(N, p, mat, src, dt_coarse)

            def advance(k, traj=traj):
                traj.step_closure(rollout_net, k, gate)
        fine = _solver(N, p, mat, src, dt_fine)
        coarse = _solver(N, p, mat, src, dt_coarse)
        advance(warmup)
        for _ in range(pairs_per_map):
            coarse.copy_state_from(traj)
            fine.copy_state_from(traj)
            coarse.closure_mark()
            coarse.step(1)
            fine.step(fine_sub)
            x = torch.empty((D, N_FEATURES), dtype=torch.float32, device="cuda")
            t = torch.empty((D, N_OUTPUTS), dtype=torch.float32, device="cuda")
            s = torch.empty(1, dtype=torch.float32, device="cuda")
            coarse.closure_features(x, s)
            coarse.closure_target(fine, s, t)
            pairs.x.append(x)
            pairs.t.append(t)
            advance(every)
        for sv in (traj, fine, coarse):
            sv.sync()
            sv.close()
    return pairs


def train(net: Network, pairs: PairSet, iters: int, lr: float = 2e-3, lr_final: float = 1e-4,
          seed: int = 0, log_every: int = 0, log=print) -> List[float]:
    """Adam on the mean squared error, one random pair per iteration, cosine
    learning-rate decay from lr to lr_final.  Returns the per-iteration loss
    (read back every log_every iterations, else only at the end)."""
    import torch

    rng = np.random.default_rng(seed)
    y = torch.empty_like(pairs.t[0])
    dy = torch.empty_like(pairs.t[0])
    losses = []
    for it in range(iters):
        k = int(rng.integers(len(pairs.x)))
        net.forward(pairs.x[k], pairs.grid, y)
        want = (log_every and (it % log_every == 0)) or it == iters - 1
        loss, _ = net.mse(y, pairs.t[k], dy, want_loss=bool(want))
        net.backward(dy)
        frac = it / max(1, iters - 1)
        cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
        net.adam(cur)
        if want:
            losses.append((it, loss))
            if log_every:
                log(f"iter {it:5d}  loss {loss:.4e}  lr {cur:.2e}")
    return losses


def evaluate_loss(net: Network, pairs: PairSet) -> float:
    """Mean loss of the network over a pair set, and of the zero correction."""
    import torch

    y = torch.empty_like(pairs.t[0])
    dy = torch.empty_like(pairs.t[0])
    tot = 0.0
    for x, t in zip(pairs.x, pairs.t):
        net.forward(x, pairs.grid, y)
        loss, _ = net.mse(y, t, dy)
        tot += loss
    return tot / len(pairs.x)


def target_energy(pairs: PairSet) -> float:
    """Mean squared target: the loss of the zero correction."""
    return float(sum(float((t.double() ** 2).mean()) for t in pairs.t) / len(pairs.t))


# ------------------------------------------------------------- evaluation
def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """Relative l2 distance of two coefficient vectors."""
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_comparison(N: int, p: int, material, source, dt_fine: float, fine_steps: int,
                   net: Network, ratio: int = 4, ref_sub: int = 4, gate: float = 0.0,
                   time_reps: int = 1) -> dict:
    """Plain ADI at dt_fine, plain ADI at ratio*dt_fine, closure at
    ratio*dt_fine, all against float64 ADI at dt_fine/ref_sub, from a zero
    state over fine_steps fine steps.  Times are per run, on the GPU, with
    HIP events (best of time_reps)."""
    import torch

    assert fine_steps % ratio == 0
    out = {}
    ref = _solver(N, p, material, source, dt_fine / ref_sub)
    ref.step(fine_steps * ref_sub)
    uref, tref = ref.get_fields()
    ref.close()

    def timed(name, run):
        best = None
        for _ in range(time_reps):
            s0 = torch.cuda.Event(enable_timing=True)
            s1 = torch.cuda.Event(enable_timing=True)
            solver = run(None)
            torch.cuda.synchronize()
            s0.record()
            run(solver)
            s1.record()
            torch.cuda.synchronize()
            ms = s0.elapsed_time(s1)
            best = ms if best is None else min(best, ms)
            u, t = solver.get_fields()
            if solver is not None and name == "closure":
                out["rejected"] = solver.closure_rejected()
            solver.close()
        return u, t, best

    def plain(dt, steps):
        def run(solver):
            if solver is None:
                return _solver(N, p, material, source, dt)
            solver.step(steps)
        return run

    def closure_run(solver):
        if solver is None:
            return _solver(N, p, material, source, dt_fine * ratio)
        solver.step_closure(net, fine_steps // ratio, gate)

    for name, run in (("fine", plain(dt_fine, fine_steps)),
                      ("coarse", plain(dt_fine * ratio, fine_steps // ratio)),
                      ("closure", closure_run)):
        u, t, ms = timed(name, run)
        out[name] = dict(rel_l2=rel_l2(u, uref), ms=ms, t_end=t)
    out["ref_t_end"] = tref
    out["speedup_vs_fine"] = out["fine"]["ms"] / out["closure"]["ms"]
    return out

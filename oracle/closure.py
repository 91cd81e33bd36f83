"""Float64 reference of the learned closure network (oracle, test only).

The paper has no learned component; this is the reference for the small 3D
convolutional network that corrects the splitting error of a coarse ADI
step.  Architecture: three 3x3x3 convolutions with zero padding on a
channels-last grid (z, y, x, c): cin -> hidden (SiLU) -> hidden (SiLU) ->
cout.  Weights W[l] have shape (27, cin_l, cout_l), tap index
t = 9 tz + 3 ty + tx, and the layer computes
    out[v, o] = b[o] + sum_t sum_i in[v + (tz-1, ty-1, tx-1), i] W[t, i, o].
Everything here is the plain definition: explicit sums over the 27 offsets.
"""
from __future__ import annotations

import numpy as np

TAPS = [(tz, ty, tx) for tz in range(3) for ty in range(3) for tx in range(3)]


def shift(x: np.ndarray, tz: int, ty: int, tx: int) -> np.ndarray:
    """y[z, y, x] = x[z + tz - 1, y + ty - 1, x + tx - 1] (zero outside)."""
    nz, ny, nx = x.shape[:3]
    out = np.zeros_like(x)
    dz, dy, dx = tz - 1, ty - 1, tx - 1
    zs = slice(max(0, -dz), min(nz, nz - dz))
    ys = slice(max(0, -dy), min(ny, ny - dy))
    xs = slice(max(0, -dx), min(nx, nx - dx))
    zt = slice(zs.start + dz, zs.stop + dz)
    yt = slice(ys.start + dy, ys.stop + dy)
    xt = slice(xs.start + dx, xs.stop + dx)
    out[zs, ys, xs] = x[zt, yt, xt]
    return out


def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3x3 convolution (cross-correlation), zero padding, channels last."""
    out = np.zeros(x.shape[:3] + (W.shape[2],))
    for t, (tz, ty, tx) in enumerate(TAPS):
        out += shift(x, tz, ty, tx) @ W[t]
    return out + b


def conv3_backward(x: np.ndarray, W: np.ndarray, dout: np.ndarray):
    """Gradients of conv3 w.r.t. its input, weights and bias."""
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    for t, (tz, ty, tx) in enumerate(TAPS):
        xs = shift(x, tz, ty, tx)
        dW[t] = np.einsum("zyxi,zyxo->io", xs, dout)
        # the adjoint of the shift by (t-1) is the shift by (1-t)
        dx += shift(dout @ W[t].T, 2 - tz, 2 - ty, 2 - tx)
    db = dout.sum(axis=(0, 1, 2))
    return dx, dW, db


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """params = [(W1,b1), (W2,b2), (W3,b3)]; returns (y, cache)."""
    (W1, b1), (W2, b2), (W3, b3) = params
    z1 = conv3(x, W1, b1)
    a1 = silu(z1)
    z2 = conv3(a1, W2, b2)
    a2 = silu(z2)
    y = conv3(a2, W3, b3)
    return y, (x, z1, a1, z2, a2)


def backward(params, cache, dy):
    """Parameter gradients for the loss gradient dy (same shape as y)."""
    (W1, b1), (W2, b2), (W3, b3) = params
    x, z1, a1, z2, a2 = cache
    da2, dW3, db3 = conv3_backward(a2, W3, dy)
    dz2 = da2 * silu_grad(z2)
    da1, dW2, db2 = conv3_backward(a1, W2, dz2)
    dz1 = da1 * silu_grad(z1)
    _, dW1, db1 = conv3_backward(x, W1, dz1)
    return [(dW1, db1), (dW2, db2), (dW3, db3)]


def mse(y, target):
    """Mean squared error over all entries and its gradient."""
    r = y - target
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unflatten(flat, shapes):
    """shapes = [(cin, cout), ...] per layer -> [(W, b), ...]."""
    out, o = [], 0
    for cin, cout in shapes:
        W = flat[o:o + 27 * cin * cout].reshape(27, cin, cout)
        o += 27 * cin * cout
        b = flat[o:o + cout]
        o += cout
        out.append((W, b))
    return out


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float values to bfloat16 (round to nearest even), as float64.

    The standard bit manipulation of IEEE single precision: bfloat16 keeps
    the upper 16 bits of a float32, and adding 0x7FFF plus the lowest kept
    bit before truncating rounds to nearest with ties to even (the rounding
    of the bfloat16 format's conversion, as in e.g. Intel's BFLOAT16
    hardware numerics definition, 2018)."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# Solver-side glue of the closure (plain definitions, float64).  States are
# (6, n, n, n) arrays [E1, E2, E3, H1, H2, H3] in [z][y][x] order; network
# tensors are channels last.
# --------------------------------------------------------------------------
N_FEATURES = 16


def closure_scale(C: np.ndarray) -> float:
    """RMS of a state over all its 6 n^3 values."""
    return float(np.sqrt(np.mean(C * C)))


def closure_features(problem, C: np.ndarray, S: np.ndarray, t_after: float):
    """Network inputs of one coarse step from S (before) to C (after).

    Channels: C / s (6), (C - S) / s (6), log eps, log mu, c / (1 + c) with
    the conductivity number c = sigma dt / (4 eps), and the dipole's impulse
    over the step, dt/2 (J(t - 3dt/4) + J(t - dt/4)) with J the source's
    coefficient field (the substep midpoints of the scheme), divided by s.
    Returns (x, s).
    """
    from . import maxwell

    n, dt = problem.n, problem.dt
    s = closure_scale(C)
    x = np.zeros((n, n, n, N_FEATURES))
    for c in range(6):
        x[..., c] = C[c] / s
        x[..., 6 + c] = (C[c] - S[c]) / s
    cc = problem.sig * dt / (4.0 * problem.eps)
    x[..., 12] = np.log(problem.eps)
    x[..., 13] = np.log(problem.mu)
    x[..., 14] = cc / (1.0 + cc)
    src = problem.source
    if src is not None and src.amp != 0.0:
        J = problem.source_rows(src.comp, t_after - 0.75 * dt) + \
            problem.source_rows(src.comp, t_after - 0.25 * dt)
        x[..., 15] = 0.5 * dt * J / s
    return x, s


def closure_target(F: np.ndarray, C: np.ndarray, s: float) -> np.ndarray:
    """(F - C) / s channels last: the correction the network learns."""
    return np.moveaxis((F - C) / s, 0, -1)


def closure_apply(C: np.ndarray, y: np.ndarray, s: float) -> np.ndarray:
    """C + s y on every coefficient that the PEC condition leaves free."""
    from . import maxwell

    out = C.copy()
    for c in range(6):
        kind, comp = ("E", c) if c < 3 else ("H", c - 3)
        out[c] += maxwell.zero_boundary(s * y[..., c], maxwell.dirichlet_axes(kind, comp))
    return out

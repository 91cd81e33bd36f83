"""Pins of the float64 closure-network oracle (CPU only): library routines
(torch CPU conv3d, autograd, Adam, bfloat16 conversion) and central finite
differences."""
import numpy as np
import pytest

from oracle import closure as C
from oracle import closure as oc

torch = pytest.importorskip("torch")


def _params(shapes, seed):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((27, ci, co)) / np.sqrt(27 * ci), 0.1 * rng.standard_normal(co))
            for ci, co in shapes]


SHAPES = [(5, 8), (8, 8), (8, 3)]


def _torch_conv(x, W, b):
    xt = torch.tensor(x).permute(3, 0, 1, 2)[None]           # N C D H W
    Wt = torch.tensor(W).reshape(3, 3, 3, W.shape[1], W.shape[2]).permute(4, 3, 0, 1, 2)
    y = torch.nn.functional.conv3d(xt, Wt, torch.tensor(b), padding=1)
    return y[0].permute(1, 2, 3, 0).numpy()


def test_conv3_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 6, 7, 4))
    W = rng.standard_normal((27, 4, 3))
    b = rng.standard_normal(3)
    np.testing.assert_allclose(C.conv3(x, W, b), _torch_conv(x, W, b), rtol=1e-12, atol=1e-12)


def test_network_forward_backward_match_autograd():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 5, 6, 5))
    params = _params(SHAPES, 2)
    y, cache = C.forward(params, x)
    target = rng.standard_normal(y.shape)
    loss, dy = C.mse(y, target)
    grads = C.backward(params, cache, dy)

    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]

    def tconv(a, W, b):
        at = a.permute(3, 0, 1, 2)[None]
        Wt = W.reshape(3, 3, 3, W.shape[1], W.shape[2]).permute(4, 3, 0, 1, 2)
        return torch.nn.functional.conv3d(at, Wt, b, padding=1)[0].permute(1, 2, 3, 0)

    a = torch.tensor(x)
    a = torch.nn.functional.silu(tconv(a, *tp[0]))
    a = torch.nn.functional.silu(tconv(a, *tp[1]))
    yt = tconv(a, *tp[2])
    lt = torch.mean((yt - torch.tensor(target)) ** 2)
    lt.backward()
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    for (gW, gb), (W, b) in zip(grads, tp):
        np.testing.assert_allclose(gW, W.grad.numpy(), rtol=1e-10, atol=1e-14)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_gradient_central_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((3, 4, 4, 5))
    params = _params(SHAPES, 4)
    target = rng.standard_normal((3, 4, 4, 3))
    flat = C.flatten(params)

    def loss_of(f):
        y, _ = C.forward(C.unflatten(f, SHAPES), x)
        return C.mse(y, target)[0]

    y, cache = C.forward(params, x)
    g = C.flatten(C.backward(params, cache, C.mse(y, target)[1]))
    idx = rng.choice(flat.size, 40, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        fd = (loss_of(flat + e) - loss_of(flat - e)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-6, abs=1e-9)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p = p0.copy()
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = C.adam(p, g, m, v, t, 3e-3)
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(6)
    a = rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000)
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(C.bf16_round(a), ref)


# ---------------------------------------------------------------- glue
def _glue_problem(seed=0, N=4, p=2, with_source=True):
    import workloads
    from oracle import maxwell
    mat = workloads.random_material(4, seed)
    src = workloads.DipoleSource(xs=(0.37, 0.52, 0.61)) if with_source else None
    return maxwell.problem_from_voxels(N, p, mat, 0.05, src)


def test_features_invariant_under_state_scaling():
    pb = _glue_problem()
    rng = np.random.default_rng(7)
    S = rng.standard_normal((6,) + (pb.n,) * 3)
    C = S + 0.1 * rng.standard_normal(S.shape)
    x1, s1 = closure_feats(pb, C, S)
    x2, s2 = closure_feats(pb, 3.0 * C, 3.0 * S)
    assert s2 == pytest.approx(3.0 * s1, rel=1e-14)
    np.testing.assert_allclose(x2[..., :12], x1[..., :12], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(x2[..., 15], x1[..., 15] / 3.0, rtol=1e-13, atol=1e-18)
    # the RMS normalised state has unit mean square
    assert np.mean(x1[..., :6] ** 2) == pytest.approx(1.0, rel=1e-13)
    # C == S: the difference channels vanish
    x3, _ = closure_feats(pb, C, C)
    assert np.all(x3[..., 6:12] == 0.0)


def closure_feats(pb, state, prev, t_after=0.55):
    return oc.closure_features(pb, state, prev, t_after)


def test_source_channel_is_the_impulse_of_the_step():
    """Partition of unity of the B-splines: summing the source channel over
    all coefficients leaves the time impulse, which is the integral of the
    dipole's time profile over the step up to the midpoint rule's O(dt^3)."""
    from scipy.integrate import quad
    from oracle import maxwell
    pb = _glue_problem()
    rng = np.random.default_rng(8)
    C = rng.standard_normal((6,) + (pb.n,) * 3)
    for t_after in (0.35, 0.5, 0.62):
        x, s = closure_feats(pb, C, C, t_after)
        impulse = x[..., 15].sum() * s
        exact = quad(lambda t: maxwell.source_time(t, pb.source), t_after - pb.dt, t_after,
                     epsabs=1e-14)[0] * pb.source.amp
        # midpoint rules on two halves: |error| <= dt^3 max|g''| / 96
        g2 = (2 * np.pi * pb.source.f0) ** 2 + 6 / pb.source.width ** 2
        assert abs(impulse - exact) <= pb.dt ** 3 * g2 / 96 * 1.01
        assert abs(impulse) > 0.1 * abs(exact) or abs(exact) < 1e-4
    # no source: the channel is zero
    pb0 = _glue_problem(with_source=False)
    x0, _ = closure_feats(pb0, C, C, 0.5)
    assert np.all(x0[..., 15] == 0.0)


def test_material_channels():
    pb = _glue_problem(seed=3)
    rng = np.random.default_rng(9)
    C = rng.standard_normal((6,) + (pb.n,) * 3)
    x, _ = closure_feats(pb, C, C)
    np.testing.assert_allclose(np.exp(x[..., 12]), pb.eps, rtol=1e-13)
    np.testing.assert_allclose(np.exp(x[..., 13]), pb.mu, rtol=1e-13)
    # c/(1+c) lies in [0, 1) and increases with sigma
    assert np.all((x[..., 14] >= 0) & (x[..., 14] < 1))
    cnum = pb.sig * pb.dt / (4 * pb.eps)
    np.testing.assert_allclose(x[..., 14] / (1 - x[..., 14]), cnum, rtol=1e-12, atol=1e-15)


def test_apply_keeps_pec_coefficients_and_inverts_target():
    from oracle import closure
    pb = _glue_problem()
    n = pb.n
    rng = np.random.default_rng(10)
    C = rng.standard_normal((6, n, n, n))
    F = rng.standard_normal((6, n, n, n))
    s = closure.closure_scale(C)
    y = closure.closure_target(F, C, s)
    out = closure.closure_apply(C, y, s)
    # brute force over the coefficients: PEC fixes E_c on the faces normal
    # to the other two axes and H_c on the faces normal to axis c
    for c in range(6):
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    on = [i in (0, n - 1), j in (0, n - 1), k in (0, n - 1)]
                    comp = c % 3
                    fixed = any(on[a] for a in range(3) if a != comp) if c < 3 else on[comp]
                    want = C[c, k, j, i] if fixed else F[c, k, j, i]
                    assert out[c, k, j, i] == pytest.approx(want, rel=1e-13, abs=1e-13)

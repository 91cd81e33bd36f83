"""Pins of the float64 closure-network oracle (CPU only): library routines
(torch CPU conv3d, autograd, Adam, bfloat16 conversion) and central finite
differences."""
import numpy as np
import pytest

from oracle import closure as C

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

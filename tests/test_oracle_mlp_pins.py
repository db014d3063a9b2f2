"""Pins of the MLP oracle (oracle/mlp.py) against things other than itself:
a closed form for the forward pass, central differences for the backward
pass, torch's bfloat16 conversion for the rounding and torch.optim.Adam for
the optimiser step.  CPU only."""
import numpy as np
import pytest
import torch

from oracle import mlp

IN = 22
SHAPES = mlp.shapes(IN)
NPARAM = mlp.nparam(IN)

rng = np.random.default_rng(0)


def rand_params(seed=1, scale=1.0):
    r = np.random.default_rng(seed)
    out = []
    for s in SHAPES:
        fan = s[-1] if len(s) == 2 else 1
        out.append(r.uniform(-1, 1, size=s) * scale / np.sqrt(max(fan, 1)))
    return mlp.pack(out)


NORM = (np.zeros(22), np.ones(22), 1.0)


def test_bf16_matches_torch():
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(
        -8, 8, size=20000), [0.0, -0.0, 1.0, 65504.0, 1e-40, 3.0e38]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(
        torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def test_param_count():
    assert NPARAM == 52609


def test_forward_closed_form_chain():
    # route input 0 through unit 0 of every layer with weight 1, zero
    # biases, output weight w and bias c: y = w * silu^4(x0) + c
    ws = [np.zeros(s) for s in SHAPES]
    for l in range(mlp.LAYERS):
        ws[2 * l][0, 0] = 1.0
    ws[8][0, 0] = 0.75
    ws[9][0] = -0.25
    p = mlp.pack(ws)
    x = np.zeros((5, 22))
    x[:, 0] = [-2.0, -0.5, 0.0, 0.7, 3.0]
    y, _ = mlp.forward(p, x, *NORM, rounding=False)
    s = x[:, 0]
    for _ in range(4):
        s = s / (1.0 + np.exp(-s))
    np.testing.assert_allclose(y, 0.75 * s - 0.25, rtol=1e-14, atol=1e-15)
    # normalisation and output scale enter as an affine map
    off, sc = np.full(22, 0.5), np.full(22, 2.0)
    y2, _ = mlp.forward(p, x, off, sc, 3.0, rounding=False)
    s = (x[:, 0] - 0.5) * 2.0
    for _ in range(4):
        s = s / (1.0 + np.exp(-s))
    np.testing.assert_allclose(y2, 3.0 * (0.75 * s - 0.25), rtol=1e-14)


def test_backward_matches_central_differences():
    p = rand_params(3)
    x = rng.normal(size=(6, 22))
    off, sc, osc = rng.normal(size=22) * 0.1, 1.0 + rng.random(22), 1.7
    dy = rng.normal(size=6)
    g, gx = mlp.backward(p, x, dy, off, sc, osc, rounding=False)

    def L(pp, xx):
        y, _ = mlp.forward(pp, xx, off, sc, osc, rounding=False)
        return float(np.dot(y, dy))
    eps = 1e-6
    idx = np.concatenate([rng.choice(NPARAM, 60, replace=False),
                          [NPARAM - 1, NPARAM - 2, 0, 2816]])
    for i in idx:
        e = np.zeros(NPARAM)
        e[i] = eps
        fd = (L(p + e, x) - L(p - e, x)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i
    for n in range(6):
        for j in (0, 1, 2, 3, 21):
            e = np.zeros_like(x)
            e[n, j] = eps
            fd = (L(p, x + e) - L(p, x - e)) / (2 * eps)
            assert abs(fd - gx[n, j]) <= 1e-6 * max(1.0, abs(fd)), (n, j)


def test_rounding_changes_little():
    p = rand_params(4)
    x = rng.normal(size=(64, 22))
    y0, _ = mlp.forward(p, x, *NORM, rounding=False)
    y1, _ = mlp.forward(p, x, *NORM, rounding=True)
    assert np.max(np.abs(y1 - y0)) < 0.05 * np.max(np.abs(y0)) + 1e-3
    assert not np.array_equal(y0, y1)


@pytest.mark.parametrize("b1,b2,eps", [(0.9, 0.999, 1e-8), (0.8, 0.95, 1e-6)])
def test_adam_matches_torch(b1, b2, eps):
    p = rng.normal(size=300)
    m = np.zeros(300)
    v = np.zeros(300)
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(b1, b2), eps=eps)
    for step in range(1, 6):
        g = rng.normal(size=300)
        p, m, v = mlp.adam_step(p, g, m, v, step, 1e-2, b1, b2, eps)
        opt.zero_grad()
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12,
                                   atol=1e-14)


def test_mse_grad():
    y = rng.normal(size=10)
    t = rng.normal(size=10)
    l, g = mlp.mse_loss_grad(y, t)
    assert abs(l - np.mean((y - t) ** 2)) < 1e-15
    eps = 1e-7
    for i in range(10):
        e = np.zeros(10)
        e[i] = eps
        fd = (mlp.mse_loss_grad(y + e, t)[0] - mlp.mse_loss_grad(y - e, t)[0]) / (2 * eps)
        assert abs(fd - g[i]) < 1e-7

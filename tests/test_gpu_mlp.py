"""Surrogate MLP kernels (MFMA forward, input gradient, weight gradients,
Adam step) against the fp64 oracle with BF16 rounding emulated.

Tolerance.  Both sides round the same quantities to BF16, but the GPU
accumulates 128-term products in FP32 (relative error ~1e-6) while the
oracle uses fp64; a pre-activation that lands within that error of a BF16
rounding boundary rounds differently, which moves one activation, SiLU
derivative or backward pre-activation gradient by one BF16 unit (2^-8
relative).  Measured on the oracle itself (the same network evaluated with
FP32 instead of fp64 accumulation), these flips move outputs by up to
0.17% and input-gradient components by up to 1.7% of the RMS magnitude,
while the median difference is ~5e-8; a flip in one sample's backward
pass moves all 22 of its input-gradient components, so 5% of those
components moved by more than 1e-3 of RMS in that measurement (8.5% of the
samples carried a flip).  Weight gradients sum over the batch, which dilutes
single flips (no element moved by 1e-3 of RMS) but adds the FP32 rounding
of a sum of n sign-mixed terms: about sqrt(n) u |t| per term, i.e. about
n u = 1.2e-4 of the sum's RMS at n = 2048 (u = 2^-24); the GPU's median
there was 7e-5.  So the maximum error is bounded at 1% (outputs) and 5%
(gradients) of the reference's RMS, the median at 5e-5 (5e-4 for weight
gradients), and the share of elements off by more than 1e-3 at 2% (15% for
input gradients, whose flips move whole rows, and 10% for weight
gradients, where a unit's bias and weight gradients collect the flips of
every sample in the batch: 4.7% of one 128-element bias gradient in a
measured run): a systematic mistake (a wrong index, sign or dropped term)
moves the median by orders of magnitude more.
"""
import sys

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sg(dev):
    import paper_2201_05058_amd.surrogate as m
    return m


def rand_net(seed):
    r = np.random.default_rng(seed)
    out = []
    for s in omlp.SHAPES:
        fan = s[-1] if len(s) == 2 else 16
        out.append(r.uniform(-1, 1, size=s) * 1.5 / np.sqrt(fan))
    return omlp.pack(out).astype(np.float32)


def close(got, want, rtol_rms=1e-2, med=5e-5, frac=0.02):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    scale = np.sqrt(np.mean(want ** 2)) + 1e-30
    err = np.abs(got - want) / scale
    assert np.all(np.isfinite(got))
    assert err.max() <= rtol_rms, float(err.max())
    assert np.median(err) <= med, float(np.median(err))
    assert np.mean(err > 1e-3) <= frac, float(np.mean(err > 1e-3))


def setup(sg, dev, seed, n):
    r = np.random.default_rng(seed + 100)
    p = rand_net(seed)
    off = r.normal(size=22).astype(np.float32) * 0.1
    sc = (0.5 + r.random(22)).astype(np.float32)
    osc = 1.3
    x = r.normal(size=(n, 22)).astype(np.float32)
    net = sg.Mlp()
    net.set_params(p, off, sc, osc)
    xd = torch.from_numpy(x).to(dev)
    return net, p, off, sc, osc, x, xd


@pytest.mark.parametrize("seed,n", [(0, 1024), (1, 3000), (2, 77)])
def test_forward_and_input_gradient(sg, dev, seed, n):
    net, p, off, sc, osc, x, xd = setup(sg, dev, seed, n)
    say(f"mlp forward seed={seed} n={n}")
    y, gx = net.forward(xd)
    torch.cuda.synchronize()
    wy, _ = omlp.forward(p.astype(np.float64), x, off, sc, osc)
    wgx = omlp.input_gradient(p.astype(np.float64), x, off, sc, osc)
    close(y.cpu().numpy(), wy)
    close(gx.cpu().numpy(), wgx, rtol_rms=5e-2, frac=0.15)
    # parameters round-trip exactly
    np.testing.assert_array_equal(net.get_params(), p)
    net.close()


@pytest.mark.parametrize("seed,n", [(3, 2048), (4, 1500)])
def test_parameter_gradients(sg, dev, seed, n):
    net, p, off, sc, osc, x, xd = setup(sg, dev, seed, n)
    dy = np.random.default_rng(seed).normal(size=n).astype(np.float32)
    say(f"mlp gradients seed={seed} n={n}")
    gp, gx = net.gradients(xd, torch.from_numpy(dy).to(dev))
    torch.cuda.synchronize()
    wg, wgx = omlp.backward(p.astype(np.float64), x, dy, off, sc, osc)
    gp = gp.cpu().numpy()
    for name, a, b in zip(range(10), omlp.unpack(gp), omlp.unpack(wg)):
        close(a, b, rtol_rms=5e-2, med=5e-4, frac=0.10)
    close(gx.cpu().numpy(), wgx, rtol_rms=5e-2, frac=0.15)
    net.close()


def test_adam_step_matches_oracle(sg, dev):
    n = 2048
    net, p, off, sc, osc, x, xd = setup(sg, dev, 5, n)
    tgt = np.random.default_rng(9).normal(size=n).astype(np.float32)
    loss = torch.zeros(1, device=dev)
    net.train_step(xd, torch.from_numpy(tgt).to(dev), 1e-3, loss=loss)
    torch.cuda.synchronize()
    pd = p.astype(np.float64)
    y, _ = omlp.forward(pd, x, off, sc, osc)
    l0, dy = omlp.mse_loss_grad(y, tgt)
    g, _ = omlp.backward(pd, x, dy, off, sc, osc)
    want, _, _ = omlp.adam_step(pd, g, np.zeros_like(pd), np.zeros_like(pd),
                                1, 1e-3)
    got = net.get_params().astype(np.float64)
    # the first Adam step moves each parameter by about lr * sign(grad)
    step = got - pd
    wstep = want - pd
    agree = np.mean(np.sign(step) == np.sign(wstep))
    assert agree > 0.98, agree
    assert np.max(np.abs(step)) <= 1.01e-3
    assert abs(float(loss.cpu()[0]) - l0) <= 1e-2 * l0
    net.close()


def test_training_reduces_loss(sg, dev):
    # fit the distance to a sphere of radius 0.5 m (a smooth target)
    r = np.random.default_rng(11)
    n = 8192
    x = r.uniform(-1, 1, size=(n, 22)).astype(np.float32)
    t = (np.linalg.norm(x[:, :3], axis=1) - 0.5).astype(np.float32)
    net = sg.Mlp()
    net.set_params(sg.init_params(np.random.default_rng(0)), np.zeros(22),
                   np.ones(22), 1.0)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(t).to(dev)
    loss = torch.zeros(1, device=dev)
    hist = []
    for it in range(300):
        net.train_step(xd, td, 2e-3, loss=loss)
        if it % 50 == 0 or it == 299:
            hist.append(float(loss.cpu()[0]))
    say("loss history", hist)
    assert hist[-1] < 0.05 * hist[0]
    net.close()

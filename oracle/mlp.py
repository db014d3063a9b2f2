"""CPU oracle of the learned surrogate for sphere queries.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain numpy in fp64.

The surrogate is not in the paper: a small multilayer perceptron that maps
a query's features to a distance (oracle/surrogate.py), with its input
gradient taken by reverse mode through the network.  Network: n_in <= 32
inputs -> 4 hidden layers of 128 SiLU units -> 1 output.  Weights are
stored as fp32 masters and used in BF16; products accumulate in FP32 on
the GPU (fp64 here).  BF16 rounding (round to nearest even) is applied at
exactly the points where the GPU kernels round:
  - the normalised input, every hidden activation and the SiLU derivative
    are rounded to BF16 before they enter a product;
  - in the backward pass every pre-activation gradient is rounded to BF16
    before it enters a product.
Parameter vector layout (fp32, 49793 + 128 n_in values):
  W0[128][n_in] b0[128] W1[128][128] b1 W2[128][128] b2 W3[128][128] b3
  W4[1][128] b4[1].
Parity status: the forward pass is pinned by a closed form (a network that
routes one input through the SiLU chain), the backward pass by central
differences of the forward pass with rounding switched off, the BF16
rounding by torch's bfloat16 conversion, and the optimiser step by
torch.optim.Adam (tests/test_oracle_mlp_pins.py).
"""
from __future__ import annotations

import numpy as np

HID = 128
LAYERS = 4


def shapes(n_in: int):
    """Shapes of the parameter arrays of a network with n_in inputs."""
    return [(HID, n_in), (HID,), (HID, HID), (HID,), (HID, HID), (HID,),
            (HID, HID), (HID,), (1, HID), (1,)]


def nparam(n_in: int) -> int:
    return int(sum(np.prod(s) for s in shapes(n_in)))


def n_inputs(params) -> int:
    """n_in of a parameter vector (its length fixes it)."""
    n = np.asarray(params).size - nparam(0)
    assert n > 0 and n % HID == 0, "not a parameter vector of this network"
    return n // HID


def bf16(x, enabled: bool = True) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via fp32.  The value
    is returned in fp64.  With enabled=False the input is returned as is."""
    x = np.asarray(x, dtype=np.float64)
    if not enabled:
        return x
    f = x.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    out = np.where(nan, f, out)
    return out.astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64).reshape(-1)
    out, o = [], 0
    for s in shapes(n_inputs(p)):
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def pack(arrs):
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1)
                           for a in arrs])


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, in_offset, in_scale, out_scale, rounding=True):
    """x: [n, n_in] raw features.  Returns (y [n], cache)."""
    Ws = unpack(params)
    W = [bf16(Ws[2 * l], rounding) for l in range(LAYERS + 1)]
    b = [Ws[2 * l + 1] for l in range(LAYERS + 1)]
    u = (np.asarray(x, np.float64) - np.asarray(in_offset, np.float64)) * \
        np.asarray(in_scale, np.float64)
    a = [bf16(u, rounding)]
    d = []
    for l in range(LAYERS):
        z = a[l] @ W[l].T + b[l]
        a.append(bf16(silu(z), rounding))
        d.append(bf16(silu_prime(z), rounding))
    y = (a[LAYERS] @ W[LAYERS].T + b[LAYERS])[:, 0]
    return y * out_scale, {"W": W, "a": a, "d": d, "u": u}


def backward(params, x, dy, in_offset, in_scale, out_scale, rounding=True):
    """dy: [n] gradient of a scalar loss w.r.t. the outputs.
    Returns (grad_params [nparam], grad_x [n, n_in])."""
    _, c = forward(params, x, in_offset, in_scale, out_scale, rounding)
    W, a, d = c["W"], c["a"], c["d"]
    dyn = np.asarray(dy, np.float64) * out_scale          # d/d(raw output)
    grads = [None] * (2 * (LAYERS + 1))
    grads[2 * LAYERS] = (dyn[:, None] * a[LAYERS]).sum(0)[None, :]
    grads[2 * LAYERS + 1] = np.array([dyn.sum()])
    da = dyn[:, None] * W[LAYERS][0][None, :]              # d/d a_4
    for l in range(LAYERS - 1, -1, -1):
        dz = bf16(da * d[l], rounding)
        grads[2 * l] = dz.T @ a[l]
        grads[2 * l + 1] = dz.sum(0)
        da = dz @ W[l]
    gx = da * np.asarray(in_scale, np.float64)[None, :]
    return pack(grads), gx


def input_gradient(params, x, in_offset, in_scale, out_scale,
                   rounding=True):
    """d y / d x for every sample, [n, n_in]."""
    n = np.asarray(x).shape[0]
    _, gx = backward(params, x, np.ones(n), in_offset, in_scale, out_scale,
                     rounding)
    return gx


def mse_loss_grad(y, target):
    """Mean squared error and its gradient w.r.t. y."""
    r = np.asarray(y, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999,
              eps=1e-8):
    """One Adam update (Kingma & Ba, with bias correction).  Returns
    (params, m, v) as new arrays; `step` counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v

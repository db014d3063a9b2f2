"""Pins of the obstacle-factor oracle: on a planar field (written directly,
so trilinear interpolation is exact) the hinge, its Jacobian and the cost
have closed forms."""
import numpy as np

import scenegen
from oracle.factors import obstacle_factors


def test_planar_field_closed_form():
    g = scenegen.Grid(12, 10, 8, 0.1)
    # d(p) = p_x - 0.37 (metres), the same in both slices
    x = (np.arange(g.nx) + 0.5) * g.h
    f = np.broadcast_to((x - 0.37).astype(np.float32), g.shape_zyx)
    sdf = np.stack([f, f])
    rng = np.random.default_rng(2)
    S, J = 5, 7
    lo, hi = 0.5 * g.h, (np.array([g.nx, g.ny, g.nz]) - 0.5) * g.h
    c = rng.uniform(lo, hi, size=(S, J, 3)).astype(np.float32)
    r = rng.uniform(0.0, 0.1, size=J).astype(np.float32)
    sl = np.array([0, 1, 5, 1, 0], np.int32)   # 5 is past the horizon
    eps, sigma = 0.3, 0.05
    err, jac, cost = obstacle_factors(g, sdf, c, r, sl, eps, sigma)
    d = c[..., 0].astype(np.float64) - 0.37 - r[None, :]
    want = np.maximum(0.0, eps - d)
    assert np.allclose(err, want, atol=1e-6)
    act = want > 1e-6
    assert np.allclose(jac[act], [-1.0, 0.0, 0.0], atol=1e-5)
    assert (jac[want == 0] == 0).all()
    assert np.allclose(cost, 0.5 * ((err.astype(np.float64) / sigma) ** 2)
                       .sum(1), rtol=1e-12)

"""Oracle of the obstacle factors (test infrastructure: only tests, the
smoke check and the benchmark's CPU baseline use it).

GPMP2's obstacle factor, used by RHAP-GPMP2 with one composite field per
time index (the last field past the horizon): for support state i and
collision sphere j with centre c_ij and radius r_j, the error is the hinge
    e_ij = max(0, eps - (d_s(c_ij) - r_j)),   s = clamp(slice_i, 0, n-1),
with d the trilinear field value, its Jacobian with respect to the centre
    J_ij = -grad d_s(c_ij)  where e_ij > 0,  else 0,
and the factor's cost for the state with isotropic noise sigma
    cost_i = sum_j 0.5 * (e_ij / sigma)^2.
The hinge and gradient are exactly the sphere query's (oracle.query: fp64
interpolation, fp32 results); the cost is summed in fp64 in sphere order.
"""
from __future__ import annotations

import numpy as np

from . import query as _query


def obstacle_factors(grid, sdf, centre, radius, slices, eps, sigma):
    """centre [S, J, 3], radius [J], slices [S] -> (err [S, J] fp32,
    jac [S, J, 3] fp32, cost [S] fp64)."""
    c = np.asarray(centre, np.float32)
    S, J = c.shape[0], c.shape[1]
    r = np.broadcast_to(np.asarray(radius, np.float32), (S, J)).reshape(-1)
    s = np.repeat(np.asarray(slices, np.int32), J)
    _, grad, _, err = _query(grid, sdf, c.reshape(-1, 3), r, s,
                             hinge_eps=eps)
    err = err.reshape(S, J)
    grad = grad.reshape(S, J, 3)
    with np.errstate(invalid="ignore"):
        active = err > 0
    jac = np.where(active[..., None], -grad, np.float32(0.0)).astype(
        np.float32)
    jac[np.isnan(err)] = np.nan
    cost = np.zeros(S, np.float64)
    for i in range(S):
        acc = 0.0
        for j in range(J):
            q = float(err[i, j]) / sigma
            acc += 0.5 * q * q
        cost[i] = acc
    return err, jac, cost

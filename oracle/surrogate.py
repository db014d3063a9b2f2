"""Oracle of the surrogate sphere queries with exact fallback (test
infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it; the library never does).

Not in the paper: a learned stand-in for the obstacle factors' field
lookups (RHAP-GPMP2 section: distance and gradient of the composite field
at the collision spheres, with a hinge cost).  Definition:

  inputs: the centre c, the slice s and the humans' state (18 floats: per
        human k its position (px_k, py_k, 0) at t = 0 and its velocity
        (vx_k, vy_k, 0));
  t   = fp32(clamp(s, 0, n-1)) * fp32(dt) (one fp32 product);
  x   = the network's 22 features, a fixed transform of the inputs, all in
        fp32 in this order of operations:
          x[0:3] = c,  x[3] = t,
          per human k (x[4+6k : 10+6k]):
            qx = px_k + vx_k * t,  qy = py_k + vy_k * t   (its axis at t),
            dx = c_x - qx,  dy = c_y - qy,
            rho = sqrt(dx * dx + dy * dy)      (horizontal distance to the
                                                axis; correctly rounded),
            [dx, dy, rho, vx_k, vy_k, 0];
  y   = network(x) in metres (oracle/mlp.py), G = dy/dx (22);
  g   = dy/dc through the transform:
          g_x = G[0] + sum_k (G[4+6k] + G[6+6k] * dx_k / rho_k),
          g_y = G[1] + sum_k (G[5+6k] + G[6+6k] * dy_k / rho_k),
          g_z = G[2],
        the ratios taken as 0 where rho_k = 0, the sums in k order in fp32;
  a query with slice s < 0 returns NaN and the SLICE_NEG bit (as exact);
  it is answered exactly (oracle.query on the composite fields) when its
  centre lies outside the span of voxel centres, or when y - r is below the
  margin or y - r or g is not finite (reading: the margin applies to the
  predicted sphere distance, the conservative one of the two readings);
  otherwise dist = y - r (fp32 subtraction of the fp32 network output),
  grad = g, status = SLICE_CLAMPED when s > n-1, cost = max(0, eps - dist).

With the environment's fp32 field given, the network predicts the humans'
part only and y is replaced by min(e, y) before the rule is applied, e the
environment field at the centre as the exact query samples it (fp64
trilinear rounded to fp32, zero radius); where e <= y (ties included) the
gradient is the environment's.
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp
from . import query as _exact_query

SLICE_CLAMPED, SLICE_NEG = 8, 32


def features(centre, slices, n_slices: int, dt: float, state) -> np.ndarray:
    """The network's 22 features (module docstring), fp32."""
    c = np.asarray(centre, np.float32).reshape(-1, 3)
    s = np.clip(np.asarray(slices, np.int64).reshape(-1), 0, n_slices - 1)
    st = np.asarray(state, np.float32).reshape(-1)
    assert st.size == 18
    t = s.astype(np.float32) * np.float32(dt)
    x = np.zeros((c.shape[0], 22), np.float32)
    x[:, 0:3] = c
    x[:, 3] = t
    for k in range(3):
        px, py, vx, vy = st[6 * k], st[6 * k + 1], st[6 * k + 3], st[6 * k + 4]
        qx = px + vx * t
        qy = py + vy * t
        dx = c[:, 0] - qx
        dy = c[:, 1] - qy
        b = 4 + 6 * k
        x[:, b] = dx
        x[:, b + 1] = dy
        x[:, b + 2] = np.sqrt(dx * dx + dy * dy)
        x[:, b + 3] = vx
        x[:, b + 4] = vy
    return x


def centre_gradient(x, G) -> np.ndarray:
    """dy/dc from the feature gradient G [n, 22] (module docstring), fp32."""
    x = np.asarray(x, np.float32)
    G = np.asarray(G).astype(np.float32)
    gx, gy, gz = G[:, 0].copy(), G[:, 1].copy(), G[:, 2].copy()
    for k in range(3):
        b = 4 + 6 * k
        rho = x[:, b + 2]
        with np.errstate(invalid="ignore", divide="ignore"):
            ux = np.where(rho > 0, x[:, b] / rho, np.float32(0))
            uy = np.where(rho > 0, x[:, b + 1] / rho, np.float32(0))
        gx = gx + G[:, b]
        gx = gx + G[:, b + 2] * ux.astype(np.float32)
        gy = gy + G[:, b + 1]
        gy = gy + G[:, b + 2] * uy.astype(np.float32)
    return np.stack([gx, gy, gz], axis=1).astype(np.float32)


def in_span(grid, centre) -> np.ndarray:
    """Centre inside [first, last] voxel centre on every axis (fp64)."""
    c = np.asarray(centre, np.float32).astype(np.float64).reshape(-1, 3)
    n = np.array([grid.nx, grid.ny, grid.nz], np.float64)
    g = (c - np.asarray(grid.origin, np.float64)[None, :]) / grid.h - 0.5
    return np.all((g >= 0.0) & (g <= n[None, :] - 1.0), axis=1)


def query(grid, sdf, params, in_offset, in_scale, out_scale, state, dt,
          centre, radius, slices, margin: float, hinge_eps: float = 0.0,
          y=None, gx=None, static_sdf=None):
    """Returns (dist, grad, status, cost, used, y).  y/gx may be given to
    decide with a network output computed elsewhere (same shapes as
    oracle/mlp.py returns); by default the fp64 oracle network is used."""
    n_slices = sdf.shape[0]
    s = np.asarray(slices, np.int64).reshape(-1)
    r = np.asarray(radius, np.float32).reshape(-1)
    x = features(centre, s, n_slices, dt, state)
    if y is None:
        p = np.asarray(params, np.float64)
        y, _ = _mlp.forward(p, x, in_offset, in_scale, out_scale)
        gx = _mlp.input_gradient(p, x, in_offset, in_scale, out_scale)
    y32 = np.asarray(y).astype(np.float32).copy()
    g32 = centre_gradient(x, gx)
    if static_sdf is not None:
        e, eg, _, _ = _exact_query(
            grid, np.asarray(static_sdf, np.float32).reshape(
                (1,) + tuple(sdf.shape[1:])), centre,
            np.zeros(len(r), np.float32), np.zeros(len(r), np.int32))
        with np.errstate(invalid="ignore"):
            take = e <= y32
        y32[take] = e[take]
        g32[take] = eg[take]
    with np.errstate(invalid="ignore", over="ignore"):
        ds = y32 - r
        ok = (in_span(grid, centre) & np.isfinite(ds) & (ds >= margin) &
              np.all(np.isfinite(g32), axis=1))
    ok &= s >= 0
    used = ((s >= 0) & ~ok).astype(np.uint8)
    dist, grad, st, cost = _exact_query(grid, sdf, centre, r, s.astype(
        np.int32), hinge_eps=hinge_eps)
    dist[ok] = ds[ok]
    grad[ok] = g32[ok]
    st[ok] = np.where(s[ok] > n_slices - 1, SLICE_CLAMPED, 0)
    hc = hinge_eps - ds[ok].astype(np.float64)
    cost[ok] = np.maximum(hc, 0.0).astype(np.float32)
    return dist, grad, st, cost, used, np.asarray(y)

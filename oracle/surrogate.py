"""Oracle of the surrogate sphere queries with exact fallback (test
infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it; the library never does).

Not in the paper: a learned stand-in for the obstacle factors' field
lookups (RHAP-GPMP2 section: distance and gradient of the composite field
at the collision spheres, with a hinge cost).  Definition:

  x   = [c_x, c_y, c_z, t, state (18)],  t = fp32(clamp(s, 0, n-1)) * fp32(dt)
        (one fp32 product, as the network's input is fp32);
  y   = network(x) in metres, g = dy/d(c_x, c_y, c_z)  (oracle/mlp.py);
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
    c = np.asarray(centre, np.float32).reshape(-1, 3)
    s = np.clip(np.asarray(slices, np.int64).reshape(-1), 0, n_slices - 1)
    st = np.asarray(state, np.float32).reshape(-1)
    assert st.size == 18
    x = np.empty((c.shape[0], 22), np.float32)
    x[:, 0:3] = c
    x[:, 3] = s.astype(np.float32) * np.float32(dt)
    x[:, 4:] = st[None, :]
    return x


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
    g32 = np.asarray(gx)[:, :3].astype(np.float32).copy()
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

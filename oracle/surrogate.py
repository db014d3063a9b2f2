"""Oracle of the surrogate sphere queries with exact fallback (test
infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use it; the library never does).

Not in the paper: a learned stand-in for the obstacle factors' field
lookups (RHAP-GPMP2 section: distance and gradient of the composite field
at the collision spheres, with a hinge cost).  The composite is the min of
the environment field and the humans' field (mapping section), and outside
the humans the field of their union is the min of the single humans'
fields, so the surrogate is one network per human: it predicts the single
human's exact field at the query as d, the distance to the continuous
cylinder, plus a learned residual, and the answer is the min over the
environment field (sampled exactly) and the humans.  Definition, in voxel
units of the grid unless stated:

  fixed point (as the exact path): X = rint(((x - o_x)/h) 2^16), Y, R =
      rint((r/h) 2^16), Hq; Kt = min(floor((Hq - 2^15)/2^16), nz - 1), no
      humans when Hq < 2^15;
  query: s' = clamp(s, 0, n-1), g_a = (c_a - o_a)/h - 1/2 (fp64);
  per human k of slice s' (fp64):
      cx = X/2^16 - 1/2, cy likewise (its axis; voxel centres lie at
      integer g), Rv = R/2^16,
      ux = g_x - cx, uy = g_y - cy, rho = sqrt(ux^2 + uy^2),
      a = rho - Rv, w = g_z - Kt, d = sqrt(max(a,0)^2 + max(w,0)^2)
      (the distance to the continuous cylinder of radius Rv and top Kt),
      phi_x = ((X - 2^15) mod 2^16) / 2^16 (the axis' phase on the voxel
      lattice), phi_y likewise, f_a = g_a - floor(g_a) (the query's);
      features x (16, the fp64 values rounded to fp32):
        [ux/rho, uy/rho, a, w, d, 1/(1+d),
         sin 2pi phi_x, cos 2pi phi_x, sin 2pi phi_y, cos 2pi phi_y,
         sin 2pi f_x, cos 2pi f_x, sin 2pi f_y, cos 2pi f_y,
         sin 2pi f_z, cos 2pi f_z]   (ux/rho = uy/rho = 0 when rho = 0);
      delta = clamp(network(x), -1/2, 3/2) (the exact single-human field
      exceeds d by 0 to about one voxel);
      y_k = fp32(h (d + delta)) metres;
      dy_k/dc = fp32(dd/dg + [network(x) not clamped] sum_f G_f df/dg)
      (metres per metre: y_k carries the factor h and g = (c - o)/h - 1/2
      divides by it), G the network's input gradient, the derivatives of
      d and of the features in closed form (fp64);
      absent when cx + Rv < 0, cx - Rv > nx - 1, cy + Rv < 0 or
      cy - Rv > ny - 1 (no voxel centre of the grid within Rv along an
      axis), clipped when present and cx - Rv <= -1, cx + Rv >= nx,
      cy - Rv <= -1 or cy + Rv >= ny (its voxelised disk may reach beyond
      the grid, where the network, trained on whole disks, under-estimates
      the distance);
  environment: e, de/dc = the exact query of the static fp32 field at c
      (zero radius, fp64 trilinear, rounded to fp32);
  y = min(e, y_k of the present humans), the environment winning ties,
      then the lower human index; m2 = the second smallest candidate;
  a query with s < 0 returns NaN and SLICE_NEG (as the exact path);
  it is answered exactly (the exact query on the composite fields) when
      its centre lies outside the span of voxel centres, fp32(y - r) <
      margin, y - r or the gradient is not finite, m2 - y < band (the
      candidates' order may change inside the cell, where the min of
      trilinear samples differs from the trilinear sample of the min), or
      a clipped human's y_k <= y + band;
  otherwise dist = fp32(y - r), grad = dy/dc of the winner, status =
      SLICE_CLAMPED when s > n-1, cost = max(0, eps - dist).
Parity status: pinned in tests/test_oracle_surrogate_pins.py (the
features against brute-force geometry and finite differences, the
residual's range against the exact single-human field, the rule against
the exact path with a network that reproduces the residual exactly).
"""
from __future__ import annotations

import numpy as np

from . import mlp as _mlp
from . import query as _exact_query

SLICE_CLAMPED, SLICE_NEG = 8, 32
N_IN = 16
RES_LO, RES_HI = -0.5, 1.5


def _fixed(p, o, h):
    t = np.asarray(p, np.float64) - np.float64(o)
    t = t / np.float64(h)
    t = t * 65536.0
    return np.rint(t).astype(np.int64)


def top_layer(grid, height) -> int:
    """Kt: the highest layer whose centre lies at or under the top."""
    Hq = int(_fixed(height, 0.0, grid.h))
    if Hq < 32768:
        return -1
    return min((Hq - 32768) // 65536, grid.nz - 1)


def lattice(grid, centre):
    """g = (c - o)/h - 1/2 (fp64, [n, 3]) and whether c lies within the
    span of voxel centres."""
    c = np.asarray(centre, np.float32).astype(np.float64).reshape(-1, 3)
    g = (c - np.asarray(grid.origin, np.float64)[None, :]) / grid.h - 0.5
    n = np.array([grid.nx, grid.ny, grid.nz], np.float64)
    inside = np.all((g >= 0.0) & (g <= n[None, :] - 1.0), axis=1)
    return g, inside


def human_geometry(grid, human_xy, radius, height, g, slices, k):
    """Geometry of human k[q] of slice clamp(slices[q]) seen from g[q]."""
    xy = np.asarray(human_xy, np.float64)
    n = xy.shape[0]
    s = np.clip(np.asarray(slices, np.int64), 0, n - 1)
    k = np.asarray(k, np.int64)
    X = _fixed(xy[s, k, 0], grid.origin[0], grid.h)
    Y = _fixed(xy[s, k, 1], grid.origin[1], grid.h)
    Rv = float(_fixed(radius, 0.0, grid.h)) / 65536.0
    Kt = top_layer(grid, height)
    cx = X.astype(np.float64) / 65536.0 - 0.5
    cy = Y.astype(np.float64) / 65536.0 - 0.5
    G = {}
    G["present"] = ~((cx + Rv < 0) | (cx - Rv > grid.nx - 1) |
                     (cy + Rv < 0) | (cy - Rv > grid.ny - 1))
    G["clipped"] = G["present"] & ((cx - Rv <= -1) | (cx + Rv >= grid.nx) |
                                   (cy - Rv <= -1) | (cy + Rv >= grid.ny))
    ux = g[:, 0] - cx
    uy = g[:, 1] - cy
    rho = np.sqrt(ux * ux + uy * uy)
    a = rho - Rv
    w = g[:, 2] - Kt
    ap, wp = np.maximum(a, 0.0), np.maximum(w, 0.0)
    G.update(ux=ux, uy=uy, rho=rho, a=a, w=w, ap=ap, wp=wp,
             d=np.sqrt(ap * ap + wp * wp),
             phx=((X - 32768) % 65536).astype(np.float64) / 65536.0,
             phy=((Y - 32768) % 65536).astype(np.float64) / 65536.0)
    return G


def features(G, g, dtype=np.float32) -> np.ndarray:
    """The 16 features (module docstring), fp32 (fp64 values with
    dtype=np.float64)."""
    with np.errstate(invalid="ignore", divide="ignore"):
        ex = np.where(G["rho"] > 0, G["ux"] / G["rho"], 0.0)
        ey = np.where(G["rho"] > 0, G["uy"] / G["rho"], 0.0)
    f = g - np.floor(g)
    cols = [ex, ey, G["a"], G["w"], G["d"], 1.0 / (1.0 + G["d"]),
            np.sin(np.pi * (2.0 * G["phx"])), np.cos(np.pi * (2.0 * G["phx"])),
            np.sin(np.pi * (2.0 * G["phy"])), np.cos(np.pi * (2.0 * G["phy"]))]
    for a in range(3):
        cols += [np.sin(np.pi * (2.0 * f[:, a])), np.cos(np.pi * (2.0 * f[:, a]))]
    return np.stack(cols, axis=1).astype(dtype)


def value_and_gradient(G, g, h, delta, Gf):
    """y_k (fp32 metres) and dy_k/dc (fp32 [n, 3]) from the network's value
    delta [n] and input gradient Gf [n, 16] (module docstring)."""
    dl = np.asarray(delta, np.float32).astype(np.float64)
    Gf = np.asarray(Gf, np.float32).astype(np.float64)
    with np.errstate(invalid="ignore"):
        clamped = ~((dl >= RES_LO) & (dl <= RES_HI))
        dc = np.where(np.isnan(dl), dl, np.clip(dl, RES_LO, RES_HI))
    y = (h * (G["d"] + dc)).astype(np.float32)
    rho, ux, uy, d = G["rho"], G["ux"], G["uy"], G["d"]
    with np.errstate(invalid="ignore", divide="ignore"):
        ex = np.where(rho > 0, ux / rho, 0.0)
        ey = np.where(rho > 0, uy / rho, 0.0)
        dd = np.stack([np.where(d > 0, G["ap"] * ex / d, 0.0),
                       np.where(d > 0, G["ap"] * ey / d, 0.0),
                       np.where(d > 0, G["wp"] / d, 0.0)], axis=1)
        r3 = rho * rho * rho
        q00 = np.where(rho > 0, uy * uy / r3, 0.0)
        q01 = np.where(rho > 0, -ux * uy / r3, 0.0)
        q11 = np.where(rho > 0, ux * ux / r3, 0.0)
    s5 = -1.0 / ((1.0 + d) * (1.0 + d))
    net = np.zeros_like(dd)
    net[:, 0] = Gf[:, 0] * q00 + Gf[:, 1] * q01 + Gf[:, 2] * ex + \
        (Gf[:, 4] + Gf[:, 5] * s5) * dd[:, 0]
    net[:, 1] = Gf[:, 0] * q01 + Gf[:, 1] * q11 + Gf[:, 2] * ey + \
        (Gf[:, 4] + Gf[:, 5] * s5) * dd[:, 1]
    net[:, 2] = Gf[:, 3] + (Gf[:, 4] + Gf[:, 5] * s5) * dd[:, 2]
    f = g - np.floor(g)
    for a in range(3):
        net[:, a] += 2.0 * np.pi * (Gf[:, 10 + 2 * a] *
                                    np.cos(np.pi * (2.0 * f[:, a])) -
                                    Gf[:, 11 + 2 * a] *
                                    np.sin(np.pi * (2.0 * f[:, a])))
    t = dd + np.where(clamped[:, None], 0.0, net)
    return y, t.astype(np.float32)


def network(params, in_offset, in_scale, out_scale):
    """The fp64 oracle network as a function (x, k) -> (value, input
    gradient) of the rows x of human k."""
    p = np.asarray(params, np.float64)

    def run(x, k=None):
        y, _ = _mlp.forward(p, x, in_offset, in_scale, out_scale)
        gx = _mlp.input_gradient(p, x, in_offset, in_scale, out_scale)
        return y, gx
    return run


def query(grid, sdf, static_sdf, net, human_xy, radius, height, centre,
          sphere_radius, slices, margin: float, band: float,
          hinge_eps: float = 0.0):
    """Returns (dist, grad, status, cost, used).  sdf: the composite fp32
    fields [n_slices, nz, ny, nx] (for the exact answers); static_sdf: the
    environment's fp32 field; net: (x [Q, 16], k) -> (value [Q],
    gradient [Q, 16]) for the rows of human k (every query's row; only
    present humans' rows are used)."""
    xy = np.asarray(human_xy, np.float64)
    n_slices, K = xy.shape[0], xy.shape[1]
    s = np.asarray(slices, np.int64).reshape(-1)
    r = np.asarray(sphere_radius, np.float32).reshape(-1)
    Q = s.size
    g, inside = lattice(grid, centre)
    e, eg, _, _ = _exact_query(
        grid, np.asarray(static_sdf, np.float32).reshape(
            (1,) + grid.shape_zyx), centre, np.zeros(Q, np.float32),
        np.zeros(Q, np.int32))
    y = e.astype(np.float32).copy()
    gr = eg.astype(np.float32).copy()
    m2 = np.full(Q, np.inf, np.float32)
    cmin = np.full(Q, np.inf, np.float32)
    Kt = top_layer(grid, height)
    for k in range(K if Kt >= 0 else 0):
        G = human_geometry(grid, xy, radius, height, g, s,
                           np.full(Q, k, np.int64))
        x = features(G, g)
        val, gx = net(x, k)
        yk, gk = value_and_gradient(G, g, grid.h, val, gx)
        pres = G["present"]
        with np.errstate(invalid="ignore"):
            cmin = np.where(pres & G["clipped"], np.fmin(cmin, yk), cmin)
            win = pres & (yk < y)
            sec = pres & ~win & (yk < m2)
        m2 = np.where(win, y, np.where(sec, yk, m2))
        gr = np.where(win[:, None], gk, gr)
        y = np.where(win, yk, y)
    with np.errstate(invalid="ignore", over="ignore"):
        ds = (y - r).astype(np.float32)
        ok = (inside & np.isfinite(ds) & (ds >= np.float32(margin)) &
              np.all(np.isfinite(gr), axis=1) &
              ~(m2.astype(np.float64) - y.astype(np.float64) < band) &
              ~(cmin.astype(np.float64) <= y.astype(np.float64) + band))
    ok &= s >= 0
    used = ((s >= 0) & ~ok).astype(np.uint8)
    dist, grad, st, cost = _exact_query(grid, sdf, centre, r,
                                        s.astype(np.int32),
                                        hinge_eps=hinge_eps)
    dist[ok] = ds[ok]
    grad[ok] = gr[ok]
    st[ok] = np.where(s[ok] > n_slices - 1, SLICE_CLAMPED, 0)
    hc = hinge_eps - ds[ok].astype(np.float64)
    cost[ok] = np.maximum(hc, 0.0).astype(np.float32)
    return dist, grad, st, cost, used

"""Oracle of the compute-once-and-shift composite (test infrastructure:
only tests, the smoke check and the benchmark's CPU baseline use it).

Mapping section: each moving obstacle's distance field is a primitive's
field computed once, and the composite at a slice is the min of the
environment field and the obstacles' fields placed at their predicted
positions.  Placing a field on a voxel grid means shifting it by a whole
number of voxels.  Definition (every integer exact):

  - per human k, the fixed-point first-slice centre X0 = rint(((x0 - o)/h)
    * 2^16) (and Y0), its anchor voxel a = floor(X0 / 2^16), and a window
    of (2 A_x + 1) x (2 A_y + 1) x nz voxels, A = n + m, m = floor(R / 2^16)
    + 2, in which the cylinder sits at fixed-point X0 - 2^16 (a - A_x);
    the template is the signed squared EDT of that single cylinder in the
    window (a full 3-D EDT, computed once);
  - at slice s the template is shifted by d = floor((X_s - X0 + 2^15) /
    2^16) voxels (the nearest whole-voxel displacement, ties upward), so
    grid voxel i reads window voxel i - (a + d - A_x);
  - the composite is min(static SSQ, min over humans of the shifted
    templates), a human contributing nothing (+INT32_MAX) where its window
    does not reach.
"""
from __future__ import annotations

import numpy as np

from . import signed_sq, to_float

INF = np.int32(2 ** 31 - 1)


def _fixed(p, o, h) -> int:
    t = np.float64(p) - np.float64(o)
    t = t / np.float64(h)
    t = t * 65536.0
    return int(np.rint(t))


def templates(grid, xy0, radius, height):
    """Per-human windows: (templates [K][nz][Wy][Wx] int32, anchors [K][2],
    (A_x, A_y))."""
    h = grid.h
    R = _fixed(radius, 0.0, h)
    Hq = _fixed(height, 0.0, h)
    Kt = min((Hq - 32768) // 65536, grid.nz - 1) if Hq >= 32768 else -1
    m = (R >> 16) + 2
    Ax, Ay = grid.nx + m, grid.ny + m
    Wx, Wy = 2 * Ax + 1, 2 * Ay + 1
    ii = np.arange(Wx, dtype=np.int64)
    jj = np.arange(Wy, dtype=np.int64)
    out, anchors = [], []
    for x, y in np.asarray(xy0, np.float64).reshape(-1, 2):
        X0 = _fixed(x, grid.origin[0], h)
        Y0 = _fixed(y, grid.origin[1], h)
        ax, ay = X0 // 65536, Y0 // 65536
        Xp = X0 - 65536 * (ax - Ax)
        Yp = Y0 - 65536 * (ay - Ay)
        dx = 32768 * (2 * ii + 1) - Xp
        dy = 32768 * (2 * jj + 1) - Yp
        disk = (dy[:, None] ** 2 + dx[None, :] ** 2) <= R * R
        occ = np.zeros((grid.nz, Wy, Wx), np.uint8)
        if Kt >= 0:
            occ[:Kt + 1] = disk[None]
        out.append(signed_sq(occ))
        anchors.append((ax, ay, X0, Y0))
    return out, anchors, (Ax, Ay)


def template_composite(grid, static_ssq, human_xy, radius, height):
    """(int32 SSQ [n, nz, ny, nx], fp32 [n, ...]) of the definition above."""
    xy = np.asarray(human_xy, np.float64)
    n, K = xy.shape[0], xy.shape[1]
    s = np.asarray(static_ssq, np.int32)
    tm, anchors, (Ax, Ay) = templates(grid, xy[0], radius, height)
    Wy, Wx = (tm[0].shape[1], tm[0].shape[2]) if K else (0, 0)
    ii = np.arange(grid.nx)
    jj = np.arange(grid.ny)
    out = np.empty((n,) + grid.shape_zyx, np.int32)
    for sl in range(n):
        c = s.copy()
        for k in range(K):
            ax, ay, X0, Y0 = anchors[k]
            Xs = _fixed(xy[sl, k, 0], grid.origin[0], grid.h)
            Ys = _fixed(xy[sl, k, 1], grid.origin[1], grid.h)
            bx = ax + (Xs - X0 + 32768) // 65536 - Ax
            by = ay + (Ys - Y0 + 32768) // 65536 - Ay
            tu, tv = ii - bx, jj - by
            okx = (tu >= 0) & (tu < Wx)
            oky = (tv >= 0) & (tv < Wy)
            vals = np.full(grid.shape_zyx, INF, np.int32)
            sub = tm[k][:, tv[oky]][:, :, tu[okx]]
            vals[:, np.nonzero(oky)[0][:, None], np.nonzero(okx)[0][None, :]] \
                = sub
            c = np.minimum(c, vals)
        out[sl] = c
    return out, to_float(out, grid.h)

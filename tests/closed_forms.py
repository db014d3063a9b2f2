"""Closed forms of the composite at sampled voxels, valid at any grid size
(shared by the oracle pins and the GPU parity tests; independent of both).

Outside every obstacle the composite is the squared distance to the union
of the environment's inclusive index boxes and the humans' voxelised
cylinders: a minimum over boxes of clamped coordinate differences, and over
each disk's rows of (row distance)^2 + (distance to the row's chord)^2 plus
the squared distance to the cylinder's layer range.  Chords come from the
exact fixed-point disk predicate, evaluated here with Python integers.
Inside the environment and outside the humans the composite is the static
field; inside a human it is negative.
"""
import math

import numpy as np


def _fixed(p, o, h):
    return int(np.rint(((np.float64(p) - np.float64(o)) / np.float64(h))
                       * 65536.0))


def chords(X, Y, R, nx, ny):
    """Rows j of one voxelised disk, clipped to the grid, and their
    inclusive column ranges."""
    rows = []
    for j in range(ny):
        dy = 32768 * (2 * j + 1) - Y
        if dy * dy > R * R:
            continue
        w = math.isqrt(R * R - dy * dy)
        lo = max(-((-(X - w - 32768)) // 65536), 0)       # ceil
        hi = min((X + w - 32768) // 65536, nx - 1)        # floor
        if lo <= hi:
            rows.append((j, lo, hi))
    return rows


class SampledClosedForm:
    def __init__(self, sc, M=40_000, seed=0):
        g = sc.grid
        self.sc = sc
        rng = np.random.default_rng(seed)
        self.ii = rng.integers(0, g.nx, M)
        self.jj = rng.integers(0, g.ny, M)
        self.kk = rng.integers(0, g.nz, M)
        ii, jj, kk = self.ii, self.jj, self.kk
        self.flat = (kk * g.ny + jj) * g.nx + ii
        eb = np.full(M, np.iinfo(np.int64).max, np.int64)
        for i0, i1, j0, j1, k0, k1 in sc.boxes.astype(np.int64):
            d = ((ii - np.clip(ii, i0, i1)) ** 2 +
                 (jj - np.clip(jj, j0, j1)) ** 2 +
                 (kk - np.clip(kk, k0, k1)) ** 2)
            np.minimum(eb, d, out=eb)
        self.eb = eb
        self.in_static = sc.occ.reshape(-1)[self.flat] != 0
        self.R = _fixed(sc.radius, 0.0, g.h)
        Hq = _fixed(sc.height, 0.0, g.h)
        self.Kt = min((Hq - 32768) // 65536, g.nz - 1) if Hq >= 32768 else -1
        self.dz = np.maximum(kk - self.Kt, 0) ** 2

    def gather(self, field):
        """Values of a [nz, ny, nx] field (numpy or torch) at the samples."""
        try:
            import torch
            if isinstance(field, torch.Tensor):
                idx = torch.from_numpy(self.flat).to(field.device)
                return field.reshape(-1)[idx].cpu().numpy().astype(np.int64)
        except ImportError:
            pass
        return np.asarray(field).reshape(-1)[self.flat].astype(np.int64)

    def check_slice(self, j, got, ssq_static):
        sc, g = self.sc, self.sc.grid
        ii, jj, kk = self.ii, self.jj, self.kk
        eh = np.full(ii.shape, np.iinfo(np.int64).max, np.int64)
        inside_h = np.zeros(ii.shape, bool)
        for k in range(sc.n_humans):
            X = _fixed(sc.human_xy[j, k, 0], g.origin[0], g.h)
            Y = _fixed(sc.human_xy[j, k, 1], g.origin[1], g.h)
            for row, lo, hi in chords(X, Y, self.R, g.nx, g.ny):
                d = (jj - row) ** 2 + (ii - np.clip(ii, lo, hi)) ** 2
                np.minimum(eh, d, out=eh)
                inside_h |= ((jj == row) & (ii >= lo) & (ii <= hi) &
                             (kk <= self.Kt))
        eh = eh + self.dz
        free = ~self.in_static & ~inside_h
        np.testing.assert_array_equal(got[free],
                                      np.minimum(self.eb, eh)[free])
        only_static = self.in_static & ~inside_h
        np.testing.assert_array_equal(got[only_static],
                                      ssq_static[only_static])
        assert (got[inside_h] < 0).all()
        return int(free.sum()), int(inside_h.sum())

"""Seeded synthetic scenes for the predicted composite distance field.

This module only *draws inputs*: static occupancy grids made of axis-aligned
boxes, predicted human positions per time slice, and collision-sphere
queries.  It holds none of the method's arithmetic (no distance transform, no
cylinder voxelisation, no composite, no interpolation), so that the CPU
oracle and the GPU library can both consume the same inputs without sharing
any code path.

Workloads stand in for the paper's (its Oxford-IHM rooms, the robot's sphere
model and the voxel-map sizes of its composite benchmark are not public
here): room-scale grids like the 7.1 x 4.2 m arena of the dataset section,
human-sized vertical cylinders as in the mapping section, constant-velocity
predictions (the CVM baseline of the prediction section) and piecewise-linear
goal-directed paths that hold their final state (end of the prediction
section).

Every draw uses numpy's PCG64 generator with an explicit seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

__all__ = [
    "Grid", "Scene", "Queries", "draw_boxes", "voxelise_boxes",
    "cv_positions", "piecewise_positions", "draw_queries",
    "cube64", "room256", "batch64", "room512", "small_scene", "human_state",
    "HUMAN_RADIUS", "HUMAN_HEIGHT",
]

# Human primitive used throughout the paper's mapping section: a vertical
# cylinder of roughly human size.
HUMAN_RADIUS = 0.25
HUMAN_HEIGHT = 1.8


@dataclass(frozen=True)
class Grid:
    """Regular voxel grid, x fastest: idx = (k*ny + j)*nx + i.

    Voxel (i, j, k) has its centre at origin + h*(i+1/2, j+1/2, k+1/2).
    """
    nx: int
    ny: int
    nz: int
    h: float
    origin: tuple = (0.0, 0.0, 0.0)

    @property
    def shape_zyx(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nvox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def extent(self):
        return (self.nx * self.h, self.ny * self.h, self.nz * self.h)


@dataclass
class Queries:
    centre: np.ndarray   # float32 [Q, 3] metres
    radius: np.ndarray   # float32 [Q]
    slice: np.ndarray    # int32 [Q]


@dataclass
class Scene:
    name: str
    grid: Grid
    boxes: np.ndarray          # int32 [B, 6] inclusive index boxes i0,i1,j0,j1,k0,k1
    occ: np.ndarray            # uint8 [nz, ny, nx], nonzero = occupied
    human_xy: np.ndarray       # float64 [n_slices, n_humans, 2] metres
    radius: float = HUMAN_RADIUS
    height: float = HUMAN_HEIGHT
    dt: float = 0.1
    queries: Optional[Queries] = None
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_slices(self) -> int:
        return int(self.human_xy.shape[0])

    @property
    def n_humans(self) -> int:
        return int(self.human_xy.shape[1])


def draw_boxes(rng: np.random.Generator, grid: Grid, count: int,
               size_lo: float = 0.1, size_hi: float = 0.8) -> np.ndarray:
    """Axis-aligned boxes in metres, [count, 6] as (x0, x1, y0, y1, z0, z1).

    Per-axis size ~ U(size_lo, size_hi); the minimum corner ~ U(0, L - size)
    so that each box lies inside the room.  Overlaps and floating boxes are
    allowed (uniform placement in 3-D).
    """
    L = np.array(grid.extent, dtype=np.float64)
    out = np.zeros((count, 6), dtype=np.float64)
    for b in range(count):
        s = rng.uniform(size_lo, size_hi, size=3)
        s = np.minimum(s, L)
        lo = rng.uniform(0.0, 1.0, size=3) * (L - s)
        out[b, 0::2] = lo + np.asarray(grid.origin)
        out[b, 1::2] = lo + s + np.asarray(grid.origin)
    return out


def voxelise_boxes(grid: Grid, boxes_m: np.ndarray):
    """Occupancy of the voxels whose centres lie in a closed metric box.

    Returns (index_boxes int32 [B, 6] inclusive, occ uint8 [nz, ny, nx]).
    Boxes that contain no voxel centre are dropped from the index list.
    """
    o = np.asarray(grid.origin, dtype=np.float64)
    n = (grid.nx, grid.ny, grid.nz)
    occ = np.zeros(grid.shape_zyx, dtype=np.uint8)
    idx = []
    for b in boxes_m:
        lohi = []
        for a in range(3):
            lo = int(np.ceil((b[2 * a] - o[a]) / grid.h - 0.5))
            hi = int(np.floor((b[2 * a + 1] - o[a]) / grid.h - 0.5))
            lo = max(lo, 0)
            hi = min(hi, n[a] - 1)
            lohi.append((lo, hi))
        if any(lo > hi for lo, hi in lohi):
            continue
        (i0, i1), (j0, j1), (k0, k1) = lohi
        occ[k0:k1 + 1, j0:j1 + 1, i0:i1 + 1] = 1
        idx.append((i0, i1, j0, j1, k0, k1))
    return np.asarray(idx, dtype=np.int32).reshape(-1, 6), occ


def cv_positions(start_xy: np.ndarray, vel_xy: np.ndarray, n_slices: int,
                 dt: float) -> np.ndarray:
    """Constant-velocity predictions p + v*t_j with t_j = j*dt, j = 0..n-1.

    Slice 0 is the current (observed) position.  Shape [n, K, 2] float64.
    """
    t = np.arange(n_slices, dtype=np.float64) * dt
    return start_xy[None, :, :] + t[:, None, None] * vel_xy[None, :, :]


def piecewise_positions(waypoints: np.ndarray, speeds: np.ndarray,
                        n_slices: int, dt: float) -> np.ndarray:
    """Positions along time-stamped piecewise-linear paths, held at the end.

    waypoints: [K, W, 2] metres; speeds: [K, W-1] m/s per segment.  After the
    last waypoint is reached the person stays there (the paper holds the
    goal state once the estimated arrival time has passed).
    """
    K, W, _ = waypoints.shape
    out = np.zeros((n_slices, K, 2), dtype=np.float64)
    for k in range(K):
        seg = np.diff(waypoints[k], axis=0)
        seglen = np.linalg.norm(seg, axis=1)
        segt = seglen / speeds[k]
        tcum = np.concatenate([[0.0], np.cumsum(segt)])
        for j in range(n_slices):
            t = j * dt
            if t >= tcum[-1]:
                out[j, k] = waypoints[k, -1]
                continue
            s = int(np.searchsorted(tcum, t, side="right") - 1)
            s = min(max(s, 0), W - 2)
            u = (t - tcum[s]) / segt[s] if segt[s] > 0 else 0.0
            out[j, k] = waypoints[k, s] + u * seg[s]
    return out


def draw_queries(rng: np.random.Generator, grid: Grid, count: int,
                 n_slices: int, r_lo: float = 0.05, r_hi: float = 0.15,
                 slice_mode: str = "mod") -> Queries:
    """Collision spheres: centres ~ U over [h/2, L - h/2]^3 (the span of
    voxel centres), radius ~ U(r_lo, r_hi), slice = q mod n_slices."""
    L = np.array(grid.extent)
    o = np.asarray(grid.origin)
    lo = o + grid.h / 2
    hi = o + L - grid.h / 2
    c = rng.uniform(0.0, 1.0, size=(count, 3)) * (hi - lo) + lo
    r = rng.uniform(r_lo, r_hi, size=count)
    if slice_mode == "mod":
        s = np.arange(count) % max(n_slices, 1)
    else:
        s = rng.integers(0, n_slices, size=count)
    return Queries(centre=c.astype(np.float32), radius=r.astype(np.float32),
                   slice=s.astype(np.int32))


def _cv_humans(rng, grid: Grid, count: int, r: float):
    Lx, Ly, _ = grid.extent
    ox, oy, _ = grid.origin
    start = np.stack([rng.uniform(r, Lx - r, size=count) + ox,
                      rng.uniform(r, Ly - r, size=count) + oy], axis=1)
    heading = rng.uniform(0.0, 2 * np.pi, size=count)
    speed = rng.uniform(0.5, 1.5, size=count)
    vel = np.stack([speed * np.cos(heading), speed * np.sin(heading)], axis=1)
    return start, vel


def cube64(seed: int = 1) -> Scene:
    """64^3 at 0.05 m, 12 boxes, one cylinder at a seeded position, 1 slice."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = Grid(64, 64, 64, 0.05)
    boxes_m = draw_boxes(rng, g, 12)
    idx, occ = voxelise_boxes(g, boxes_m)
    Lx, Ly, _ = g.extent
    r = HUMAN_RADIUS
    xy = np.array([[[rng.uniform(r, Lx - r), rng.uniform(r, Ly - r)]]])
    return Scene("cube64", g, idx, occ, xy, dt=0.0, seed=seed)


def room256(seed: int = 2, n_queries: int = 10_000) -> Scene:
    """256x256x128 at 0.02 m, 40 boxes, 3 constant-velocity humans,
    20 slices at dt = 0.1 s, 10k sphere queries (slice = q mod 20)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = Grid(256, 256, 128, 0.02)
    boxes_m = draw_boxes(rng, g, 40)
    idx, occ = voxelise_boxes(g, boxes_m)
    start, vel = _cv_humans(rng, g, 3, HUMAN_RADIUS)
    n, dt = 20, 0.1
    xy = cv_positions(start, vel, n, dt)
    q = draw_queries(rng, g, n_queries, n)
    return Scene("room256", g, idx, occ, xy, dt=dt, queries=q, seed=seed,
                 meta={"start": start, "vel": vel})


def batch64(seed: int = 3, n_scenes: int = 64) -> List[Scene]:
    """64 independent scenes of uneven sizes: nx, ny ~ U{64..256},
    nz ~ U{64..128}, h ~ U(0.02, 0.05), boxes = max(4, round(40*vol/67.1)),
    n ~ U{5..30} slices, K ~ U{1..4} constant-velocity humans, dt = 0.1 s."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for s in range(n_scenes):
        nx = int(rng.integers(64, 257))
        ny = int(rng.integers(64, 257))
        nz = int(rng.integers(64, 129))
        h = float(rng.uniform(0.02, 0.05))
        g = Grid(nx, ny, nz, h)
        vol = float(np.prod(g.extent))
        nb = max(4, int(round(40 * vol / 67.1)))
        boxes_m = draw_boxes(rng, g, nb)
        idx, occ = voxelise_boxes(g, boxes_m)
        n = int(rng.integers(5, 31))
        K = int(rng.integers(1, 5))
        start, vel = _cv_humans(rng, g, K, HUMAN_RADIUS)
        xy = cv_positions(start, vel, n, 0.1)
        out.append(Scene(f"batch64_{s}", g, idx, occ, xy, dt=0.1, seed=seed))
    return out


def room512(seed: int = 5, queries_per_slice: int = 100_000,
            with_queries: bool = True) -> Scene:
    """512x512x256 at 0.01 m, 200 boxes, 8 humans on 4-waypoint
    piecewise-linear paths (segment speed ~ U(0.5, 1.5) m/s, held at the
    end), 50 slices at dt = 0.05 s, 100k spheres per slice."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = Grid(512, 512, 256, 0.01)
    boxes_m = draw_boxes(rng, g, 200)
    idx, occ = voxelise_boxes(g, boxes_m)
    K, W = 8, 4
    Lx, Ly, _ = g.extent
    r = HUMAN_RADIUS
    wp = np.stack([rng.uniform(r, Lx - r, size=(K, W)),
                   rng.uniform(r, Ly - r, size=(K, W))], axis=2)
    sp = rng.uniform(0.5, 1.5, size=(K, W - 1))
    n, dt = 50, 0.05
    xy = piecewise_positions(wp, sp, n, dt)
    q = None
    if with_queries:
        q = draw_queries(rng, g, queries_per_slice * n, n)
    return Scene("room512", g, idx, occ, xy, dt=dt, queries=q, seed=seed,
                 meta={"waypoints": wp, "speeds": sp})


def small_scene(seed: int, nx: int, ny: int, nz: int, h: float = 0.05,
                n_boxes: int = 6, n_humans: int = 2, n_slices: int = 3,
                dt: float = 0.2, radius: float = HUMAN_RADIUS,
                height: float = HUMAN_HEIGHT, n_queries: int = 0,
                box_hi: float = 0.8) -> Scene:
    """A small scene of arbitrary (ragged) dimensions for parity tests.

    Humans may start anywhere in (and slightly beyond) the room so that
    partial and total exits from the grid are exercised.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = Grid(nx, ny, nz, h)
    boxes_m = draw_boxes(rng, g, n_boxes, size_lo=min(0.1, box_hi / 2),
                         size_hi=box_hi)
    idx, occ = voxelise_boxes(g, boxes_m)
    Lx, Ly, _ = g.extent
    start = np.stack([rng.uniform(-radius, Lx + radius, size=n_humans),
                      rng.uniform(-radius, Ly + radius, size=n_humans)], 1)
    heading = rng.uniform(0, 2 * np.pi, size=n_humans)
    speed = rng.uniform(0.5, 1.5, size=n_humans)
    vel = np.stack([speed * np.cos(heading), speed * np.sin(heading)], 1)
    xy = cv_positions(start, vel, n_slices, dt)
    q = draw_queries(rng, g, n_queries, n_slices) if n_queries else None
    return Scene(f"small_{seed}", g, idx, occ, xy, radius=radius,
                 height=height, dt=dt, queries=q, seed=seed,
                 meta={"start": start, "vel": vel})


def human_state(start_xy: np.ndarray, vel_xy: np.ndarray) -> np.ndarray:
    """The 18 state features of three constant-velocity humans at t = 0:
    per human its position (x, y, 0) and velocity (vx, vy, 0), float32."""
    start_xy = np.asarray(start_xy, np.float64)
    vel_xy = np.asarray(vel_xy, np.float64)
    if start_xy.shape != (3, 2) or vel_xy.shape != (3, 2):
        raise ValueError("the state describes exactly three humans")
    out = np.zeros((3, 6), np.float64)
    out[:, 0:2] = start_xy
    out[:, 3:5] = vel_xy
    return out.reshape(-1).astype(np.float32)

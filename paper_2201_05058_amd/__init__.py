"""Predicted composite signed distance fields on MI355X (gfx950).

Python face of libpcsdf.so.  Each function has the name of its C-ABI
entry point (without the ``pcsdf_`` prefix), takes torch tensors that live
on the GPU, and enqueues the library's HIP kernels on torch's current
stream.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native
from ._native import (Grid, Handle, PcsdfError, Q_INF_CORNER, Q_OOR_X,
                      Q_OOR_Y, Q_OOR_Z, Q_SLICE_CLAMPED, Q_SLICE_NEG,
                      Scene, Tuning, as_grid, default_handle, load_library)

__all__ = [
    "Grid", "Handle", "PcsdfError", "build_static_sdf",
    "predicted_composite_sdf", "query_spheres", "load_library",
    "predicted_composite_sdf_growing", "recompute_sdf",
    "template_composite_sdf", "obstacle_factors", "build_floor_sdf",
    "query_spheres_direct",
    "predicted_composite_sdf_batch", "BatchGraph",
    "autotune_batch", "autotune_composite", "Scene", "Tuning",
    "Q_OOR_X", "Q_OOR_Y", "Q_OOR_Z", "Q_SLICE_CLAMPED", "Q_INF_CORNER",
    "Q_SLICE_NEG",
]


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, name, numel=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, "
                         f"got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream(device):
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def build_static_sdf(grid, occ, ssq=None, sdf=None, want_sdf=True,
                     handle: Handle | None = None):
    """Exact signed squared EDT of a uint8 occupancy grid [nz, ny, nx]
    (pcsdf_build_static_sdf).  Returns (ssq int32, sdf float32 or None)."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    V = g.nvox
    dev = occ.device
    if ssq is None:
        ssq = torch.empty(g.shape_zyx, dtype=torch.int32, device=dev)
    if sdf is None and want_sdf:
        sdf = torch.empty(g.shape_zyx, dtype=torch.float32, device=dev)
    rc = h.lib.pcsdf_build_static_sdf(
        h.ptr, C.byref(g), _dev_ptr(occ, torch.uint8, "occ", V),
        _dev_ptr(ssq, torch.int32, "ssq", V),
        _dev_ptr(sdf, torch.float32, "sdf", V), _stream(dev))
    h.check(rc)
    return ssq, sdf


def build_floor_sdf(grid, occ, z_lo=0, z_hi=None, want_sdf=True,
                    handle: Handle | None = None):
    """Signed EDT of the map collapsed to the floor plane over layers
    [z_lo, z_hi] (pcsdf_build_floor_sdf).  Returns (ssq int32 [ny, nx],
    sdf float32 [ny, nx] or None)."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    z_hi = g.nz - 1 if z_hi is None else z_hi
    dev = occ.device
    ssq = torch.empty((g.ny, g.nx), dtype=torch.int32, device=dev)
    sdf = torch.empty((g.ny, g.nx), dtype=torch.float32, device=dev) \
        if want_sdf else None
    h.check(h.lib.pcsdf_build_floor_sdf(
        h.ptr, C.byref(g), _dev_ptr(occ, torch.uint8, "occ", g.nvox),
        int(z_lo), int(z_hi), _dev_ptr(ssq, torch.int32, "ssq"),
        _dev_ptr(sdf, torch.float32, "sdf"), _stream(dev)))
    return ssq, sdf


def composite_outputs(n, shape_zyx, device, want_ssq=True, want_sdf=True):
    """Output fields [n, nz, ny, nx] (int32 squared voxel distance, fp32
    metres) as the composite calls allocate them by default: both in one
    allocation, the fp32 field starting 4 KiB past the end of the int32
    one.  Two output streams whose starts differ by a multiple of 8 KiB (as
    two separate large allocations do) write measurably more slowly on
    this GPU (256x256x128 x 20 slices: 0.239 against 0.231 ms).  The fp32
    field keeps the 16-byte alignment the widest packs need."""
    torch = _torch()
    cnt = int(n)
    for d in shape_zyx:
        cnt *= int(d)
    shp = (int(n),) + tuple(int(d) for d in shape_zyx)
    if not (want_ssq and want_sdf):
        oc = torch.empty(shp, dtype=torch.int32, device=device) \
            if want_ssq else None
        of = torch.empty(shp, dtype=torch.float32, device=device) \
            if want_sdf else None
        return oc, of
    pad = 1024  # int32 elements: 4 KiB
    buf = torch.empty(2 * cnt + pad, dtype=torch.int32, device=device)
    oc = buf[:cnt].view(shp)
    of = buf[cnt + pad:].view(torch.float32).view(shp)
    return oc, of


def predicted_composite_sdf(grid, static_ssq, human_xy, radius, height,
                            out_ssq=None, out_sdf=None, want_ssq=True,
                            want_sdf=True, handle: Handle | None = None):
    """Per-slice composite fields (pcsdf_predicted_composite_sdf).

    human_xy: host array [n_slices, n_humans, 2] of predicted positions in
    metres.  Returns (ssq int32 [n, nz, ny, nx] or None, sdf float32 or
    None)."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n, K = xy.shape[0], xy.shape[1]
    V = g.nvox
    dev = static_ssq.device
    if out_ssq is None and out_sdf is None:
        out_ssq, out_sdf = composite_outputs(n, g.shape_zyx, dev, want_ssq,
                                             want_sdf)
    shp = (n,) + g.shape_zyx
    if out_ssq is None and want_ssq:
        out_ssq = torch.empty(shp, dtype=torch.int32, device=dev)
    if out_sdf is None and want_sdf:
        out_sdf = torch.empty(shp, dtype=torch.float32, device=dev)
    rc = h.lib.pcsdf_predicted_composite_sdf(
        h.ptr, C.byref(g), _dev_ptr(static_ssq, torch.int32, "static_ssq", V),
        n, K, xy.ctypes.data_as(C.c_void_p) if K > 0 else None,
        float(radius), float(height),
        _dev_ptr(out_ssq, torch.int32, "out_ssq", n * V),
        _dev_ptr(out_sdf, torch.float32, "out_sdf", n * V), _stream(dev))
    h.check(rc)
    return out_ssq, out_sdf


def predicted_composite_sdf_noalloc(grid, static_ssq, human_xy, radius,
                                    height, out_ssq, out_sdf,
                                    handle: Handle | None = None):
    """The composite without any allocation by the library
    (pcsdf_predicted_composite_sdf_noalloc): the caller passes both output
    tensors ([n, nz, ny, nx] int32 / float32, either may be None); the
    planar fields live in the library's fixed per-device scratch."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n, K = xy.shape[0], xy.shape[1]
    V = g.nvox
    dev = static_ssq.device
    rc = h.lib.pcsdf_predicted_composite_sdf_noalloc(
        h.ptr, C.byref(g), _dev_ptr(static_ssq, torch.int32, "static_ssq", V),
        n, K, xy.ctypes.data_as(C.c_void_p) if K > 0 else None,
        float(radius), float(height),
        _dev_ptr(out_ssq, torch.int32, "out_ssq", n * V),
        _dev_ptr(out_sdf, torch.float32, "out_sdf", n * V), _stream(dev))
    h.check(rc)
    return out_ssq, out_sdf


def predicted_composite_sdf_growing(grid, static_ssq, human_xy,
                                    radius_per_slice, height, out_ssq=None,
                                    out_sdf=None, want_ssq=True,
                                    want_sdf=True,
                                    handle: Handle | None = None):
    """Composite fields with one cylinder radius per slice
    (pcsdf_predicted_composite_sdf_growing), e.g. r0 + sigma * t_j."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n, K = xy.shape[0], xy.shape[1]
    rad = np.ascontiguousarray(np.asarray(radius_per_slice, np.float64))
    if rad.shape != (n,):
        raise ValueError("radius_per_slice must have n_slices entries")
    V = g.nvox
    dev = static_ssq.device
    if out_ssq is None and out_sdf is None:
        out_ssq, out_sdf = composite_outputs(n, g.shape_zyx, dev, want_ssq,
                                             want_sdf)
    shp = (n,) + g.shape_zyx
    if out_ssq is None and want_ssq:
        out_ssq = torch.empty(shp, dtype=torch.int32, device=dev)
    if out_sdf is None and want_sdf:
        out_sdf = torch.empty(shp, dtype=torch.float32, device=dev)
    h.check(h.lib.pcsdf_predicted_composite_sdf_growing(
        h.ptr, C.byref(g), _dev_ptr(static_ssq, torch.int32, "static_ssq", V),
        n, K, xy.ctypes.data_as(C.c_void_p) if K > 0 else None,
        rad.ctypes.data_as(C.c_void_p), float(height),
        _dev_ptr(out_ssq, torch.int32, "out_ssq", n * V),
        _dev_ptr(out_sdf, torch.float32, "out_sdf", n * V), _stream(dev)))
    return out_ssq, out_sdf


def query_spheres_direct(grid, static_ssq, human_xy, radius, height, centre,
                         sphere_radius, slices, hinge_eps=0.0,
                         want_status=True, want_cost=False,
                         handle: Handle | None = None):
    """Sphere queries on the composite fields of (static_ssq, human_xy,
    radius, height) without building them (pcsdf_query_spheres_direct).
    Returns (dist, grad, status or None, cost or None) as query_spheres."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n, K = xy.shape[0], xy.shape[1]
    Q = centre.shape[0] if centre.ndim > 1 else centre.numel() // 3
    dev = static_ssq.device
    dist = torch.empty(Q, dtype=torch.float32, device=dev)
    grad = torch.empty((Q, 3), dtype=torch.float32, device=dev)
    status = (torch.empty(Q, dtype=torch.uint8, device=dev)
              if want_status else None)
    cost = torch.empty(Q, dtype=torch.float32, device=dev) if want_cost \
        else None
    h.check(h.lib.pcsdf_query_spheres_direct(
        h.ptr, C.byref(g), _dev_ptr(static_ssq, torch.int32, "static_ssq",
                                    g.nvox),
        n, K, xy.ctypes.data_as(C.c_void_p) if K > 0 else None,
        float(radius), float(height), Q,
        _dev_ptr(centre, torch.float32, "centre", 3 * Q),
        _dev_ptr(sphere_radius, torch.float32, "radius", Q),
        _dev_ptr(slices, torch.int32, "slices", Q), float(hinge_eps),
        _dev_ptr(dist, torch.float32, "dist"),
        _dev_ptr(grad, torch.float32, "grad"),
        _dev_ptr(status, torch.uint8, "status"),
        _dev_ptr(cost, torch.float32, "cost"), _stream(dev)))
    return dist, grad, status, cost


def obstacle_factors(grid, sdf, centre, radius, state_slice, eps, sigma,
                     handle: Handle | None = None):
    """GPMP2 obstacle factors of every support state
    (pcsdf_obstacle_factors): centre [S, J, 3] float32, radius [J],
    state_slice [S] int32, all on the GPU.  Returns (err [S, J],
    jac [S, J, 3], cost [S] float64)."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    V = g.nvox
    n_slices = sdf.numel() // V
    if n_slices * V != sdf.numel():
        raise ValueError("sdf size is not a whole number of fields")
    S, J = centre.shape[0], centre.shape[1]
    dev = sdf.device
    err = torch.empty((S, J), dtype=torch.float32, device=dev)
    jac = torch.empty((S, J, 3), dtype=torch.float32, device=dev)
    cost = torch.empty(S, dtype=torch.float64, device=dev)
    h.check(h.lib.pcsdf_obstacle_factors(
        h.ptr, C.byref(g), _dev_ptr(sdf, torch.float32, "sdf"), n_slices, S,
        J, _dev_ptr(centre, torch.float32, "centre", S * J * 3),
        _dev_ptr(radius, torch.float32, "radius", J),
        _dev_ptr(state_slice, torch.int32, "state_slice", S), float(eps),
        float(sigma), _dev_ptr(err, torch.float32, "err"),
        _dev_ptr(jac, torch.float32, "jac"),
        _dev_ptr(cost, torch.float64, "cost"), _stream(dev)))
    return err, jac, cost


def template_composite_sdf(grid, static_ssq, human_xy, radius, height,
                           out_ssq=None, out_sdf=None, want_ssq=True,
                           want_sdf=True, handle: Handle | None = None):
    """Compute-once-and-shift composite (pcsdf_template_composite_sdf):
    arguments and outputs as predicted_composite_sdf."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n, K = xy.shape[0], xy.shape[1]
    V = g.nvox
    dev = static_ssq.device
    if out_ssq is None and out_sdf is None:
        out_ssq, out_sdf = composite_outputs(n, g.shape_zyx, dev, want_ssq,
                                             want_sdf)
    shp = (n,) + g.shape_zyx
    if out_ssq is None and want_ssq:
        out_ssq = torch.empty(shp, dtype=torch.int32, device=dev)
    if out_sdf is None and want_sdf:
        out_sdf = torch.empty(shp, dtype=torch.float32, device=dev)
    h.check(h.lib.pcsdf_template_composite_sdf(
        h.ptr, C.byref(g), _dev_ptr(static_ssq, torch.int32, "static_ssq", V),
        n, K, xy.ctypes.data_as(C.c_void_p) if K > 0 else None,
        float(radius), float(height),
        _dev_ptr(out_ssq, torch.int32, "out_ssq", n * V),
        _dev_ptr(out_sdf, torch.float32, "out_sdf", n * V), _stream(dev)))
    return out_ssq, out_sdf


def recompute_sdf(grid, static_occ, human_xy, radius, height, out_ssq=None,
                  out_sdf=None, want_sdf=True,
                  handle: Handle | None = None):
    """Full recompute (pcsdf_recompute_sdf): the exact signed EDT of the
    environment and the humans' voxels, from scratch for every slice.
    Returns (ssq int32 [n, nz, ny, nx], sdf float32 or None)."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n, K = xy.shape[0], xy.shape[1]
    V = g.nvox
    dev = static_occ.device
    shp = (n,) + g.shape_zyx
    if out_ssq is None:
        out_ssq = torch.empty(shp, dtype=torch.int32, device=dev)
    if out_sdf is None and want_sdf:
        out_sdf = torch.empty(shp, dtype=torch.float32, device=dev)
    h.check(h.lib.pcsdf_recompute_sdf(
        h.ptr, C.byref(g), _dev_ptr(static_occ, torch.uint8, "static_occ", V),
        n, K, xy.ctypes.data_as(C.c_void_p) if K > 0 else None,
        float(radius), float(height),
        _dev_ptr(out_ssq, torch.int32, "out_ssq", n * V),
        _dev_ptr(out_sdf, torch.float32, "out_sdf", n * V), _stream(dev)))
    return out_ssq, out_sdf


class _BatchScenes:
    """pcsdf_scene array for a list of scene dicts, with outputs allocated
    where not given, and the arrays it points to kept alive."""

    def __init__(self, scenes):
        torch = _torch()
        self.keep = []
        self.outputs = []
        arr = (_native.Scene * len(scenes))()
        for q, d in enumerate(scenes):
            g = as_grid(d["grid"])
            s = d["static_ssq"]
            xy = np.ascontiguousarray(np.asarray(d["human_xy"],
                                                 dtype=np.float64))
            if xy.ndim != 3 or xy.shape[2] != 2:
                raise ValueError(f"scene {q}: human_xy must be [n, K, 2]")
            n, K = xy.shape[0], xy.shape[1]
            V = g.nvox
            shp = (n,) + g.shape_zyx
            oc = d.get("out_ssq")
            of = d.get("out_sdf")
            if oc is None and d.get("want_ssq", True):
                oc = torch.empty(shp, dtype=torch.int32, device=s.device)
            if of is None and d.get("want_sdf", True):
                of = torch.empty(shp, dtype=torch.float32, device=s.device)
            e = arr[q]
            e.grid = g
            e.static_ssq_dev = _dev_ptr(s, torch.int32, "static_ssq", V)
            e.n_slices, e.n_humans = n, K
            e.human_xy_host = xy.ctypes.data_as(C.c_void_p) if K else None
            e.radius_m = float(d["radius"])
            e.height_m = float(d["height"])
            e.out_ssq_dev = _dev_ptr(oc, torch.int32, "out_ssq", n * V)
            e.out_sdf_dev = _dev_ptr(of, torch.float32, "out_sdf", n * V)
            self.keep.append(xy)
            self.outputs.append((oc, of))
        self.arr = arr
        self.n = len(scenes)
        self.device = scenes[0]["static_ssq"].device


def predicted_composite_sdf_batch(scenes, handle: Handle | None = None):
    """All scenes in two launches, planar items then composite items
    (pcsdf_predicted_composite_sdf_batch).  `scenes` is a list of dicts
    with keys grid, static_ssq, human_xy, radius, height and optionally
    out_ssq / out_sdf / want_ssq / want_sdf.  Returns [(ssq, sdf), ...]."""
    h = handle or default_handle()
    b = _BatchScenes(scenes)
    h.check(h.lib.pcsdf_predicted_composite_sdf_batch(
        h.ptr, b.n, b.arr, _stream(b.device)))
    return b.outputs


class BatchGraph:
    """A batch captured in a hipGraph (pcsdf_batch_graph_*)."""

    def __init__(self, scenes, handle: Handle | None = None):
        self.h = handle or default_handle()
        self.b = _BatchScenes(scenes)
        g = C.c_void_p()
        self.h.check(self.h.lib.pcsdf_batch_graph_create(
            self.h.ptr, self.b.n, self.b.arr, _stream(self.b.device),
            C.byref(g)))
        self.ptr = g
        self.outputs = self.b.outputs

    def launch(self):
        self.h.check(self.h.lib.pcsdf_batch_graph_launch(
            self.ptr, _stream(self.b.device)))

    def set_positions(self, scene: int, human_xy):
        xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
        self.h.check(self.h.lib.pcsdf_batch_graph_set_positions(
            self.ptr, int(scene), xy.ctypes.data_as(C.c_void_p)))

    def close(self):
        if getattr(self, "ptr", None):
            self.h.lib.pcsdf_batch_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_batch(scenes, reps: int = 2, handle: Handle | None = None):
    """Times the batch launch shapes on these scenes and keeps the fastest
    in the handle (pcsdf_autotune_batch).  Returns (tuning dict, ms)."""
    h = handle or default_handle()
    b = _BatchScenes(scenes)
    t = _native.Tuning()
    ms = C.c_double()
    h.check(h.lib.pcsdf_autotune_batch(h.ptr, b.n, b.arr, _stream(b.device),
                                       int(reps), C.byref(t), C.byref(ms)))
    return t.as_dict(), ms.value


def autotune_composite(scene, reps: int = 3, handle: Handle | None = None):
    """Times the composite launch shapes for one scene and keeps the
    fastest in the handle (pcsdf_autotune_composite)."""
    h = handle or default_handle()
    b = _BatchScenes([scene])
    t = _native.Tuning()
    ms = C.c_double()
    h.check(h.lib.pcsdf_autotune_composite(h.ptr, b.arr, _stream(b.device),
                                           int(reps), C.byref(t),
                                           C.byref(ms)))
    return t.as_dict(), ms.value, b.outputs[0]


def query_spheres(grid, sdf, centre, radius, slices, hinge_eps=0.0,
                  want_status=True, want_cost=False,
                  handle: Handle | None = None):
    """Trilinear distance and gradient at collision spheres
    (pcsdf_query_spheres).  sdf: float32 [n_slices, nz, ny, nx] (or a
    single field [nz, ny, nx]).  Returns (dist [Q], grad [Q, 3],
    status uint8 [Q] or None, cost [Q] or None)."""
    torch = _torch()
    g = as_grid(grid)
    h = handle or default_handle()
    V = g.nvox
    n_slices = sdf.numel() // V
    if n_slices * V != sdf.numel():
        raise ValueError("sdf size is not a whole number of fields")
    Q = centre.shape[0] if centre.ndim > 1 else centre.numel() // 3
    dev = sdf.device
    dist = torch.empty(Q, dtype=torch.float32, device=dev)
    grad = torch.empty((Q, 3), dtype=torch.float32, device=dev)
    status = (torch.empty(Q, dtype=torch.uint8, device=dev)
              if want_status else None)
    cost = torch.empty(Q, dtype=torch.float32, device=dev) if want_cost \
        else None
    rc = h.lib.pcsdf_query_spheres(
        h.ptr, C.byref(g), _dev_ptr(sdf, torch.float32, "sdf"), n_slices, Q,
        _dev_ptr(centre, torch.float32, "centre", 3 * Q),
        _dev_ptr(radius, torch.float32, "radius", Q),
        _dev_ptr(slices, torch.int32, "slices", Q), float(hinge_eps),
        _dev_ptr(dist, torch.float32, "dist"),
        _dev_ptr(grad, torch.float32, "grad"),
        _dev_ptr(status, torch.uint8, "status"),
        _dev_ptr(cost, torch.float32, "cost"), _stream(dev))
    h.check(rc)
    return dist, grad, status, cost

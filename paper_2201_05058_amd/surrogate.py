"""Binding of the surrogate MLP (pcsdf_mlp_*).

The network, its gradients and its optimiser step all run in the
library's HIP kernels; this module marshals torch tensors and host arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._native import Handle, as_grid, default_handle, load_library

NIN = 16  # features per (query, human) row (PCSDF_SURROGATE_IN)
HID = 128


def shapes(n_in: int):
    return [(HID, n_in), (HID,), (HID, HID), (HID,), (HID, HID), (HID,),
            (HID, HID), (HID,), (1, HID), (1,)]


def nparam(n_in: int) -> int:
    return int(sum(np.prod(x) for x in shapes(n_in)))


def _declare(lib):
    if getattr(lib, "_mlp_declared", False):
        return
    P = C.c_void_p
    i32, f32 = C.c_int32, C.c_float
    lib.pcsdf_mlp_param_count.argtypes = [i32]
    lib.pcsdf_mlp_param_count.restype = C.c_int
    lib.pcsdf_mlp_create.argtypes = [P, i32, C.POINTER(P)]
    lib.pcsdf_mlp_create.restype = C.c_int
    lib.pcsdf_mlp_destroy.argtypes = [P]
    lib.pcsdf_mlp_destroy.restype = None
    lib.pcsdf_mlp_set_params.argtypes = [P, P, P, P, f32]
    lib.pcsdf_mlp_set_params.restype = C.c_int
    lib.pcsdf_mlp_get_params.argtypes = [P, P]
    lib.pcsdf_mlp_get_params.restype = C.c_int
    lib.pcsdf_mlp_forward.argtypes = [P, i32, P, P, P, P]
    lib.pcsdf_mlp_forward.restype = C.c_int
    lib.pcsdf_mlp_gradients.argtypes = [P, i32, P, P, P, P, P]
    lib.pcsdf_mlp_gradients.restype = C.c_int
    lib.pcsdf_mlp_train_step.argtypes = [P, i32, P, P, f32, f32, f32, f32, P,
                                         P]
    lib.pcsdf_mlp_train_step.restype = C.c_int
    lib.pcsdf_mlp_loss_gradients.argtypes = [P, i32, P, P, P, P, P]
    lib.pcsdf_mlp_loss_gradients.restype = C.c_int
    lib.pcsdf_mlp_adam_step.argtypes = [P, P, f32, f32, f32, f32, P]
    lib.pcsdf_mlp_adam_step.restype = C.c_int
    lib.pcsdf_mlp_get_state.argtypes = [P, P, P, P, C.POINTER(C.c_int64)]
    lib.pcsdf_mlp_get_state.restype = C.c_int
    lib.pcsdf_mlp_set_state.argtypes = [P, P, P, P, C.c_int64, P, P, f32]
    lib.pcsdf_mlp_set_state.restype = C.c_int
    d = C.c_double
    lib.pcsdf_surrogate_human_features.argtypes = [
        P, P, i32, i32, P, d, d, i32, P, P, P, P, P, P, P, P]
    lib.pcsdf_surrogate_human_features.restype = C.c_int
    lib.pcsdf_query_spheres_surrogate.argtypes = [
        P, P, P, P, P, i32, i32, P, d, d, d, d, i32, P, P, P, d, P, P, P, P,
        P, P, P]
    lib.pcsdf_query_spheres_surrogate.restype = C.c_int
    lib._mlp_declared = True


def init_params(rng: np.random.Generator, n_in: int = NIN) -> np.ndarray:
    """Uniform(+-1/sqrt(fan_in)) weights and biases (the numbers drawn on
    the host and passed to the library)."""
    out = []
    sh = shapes(n_in)
    for q in range(0, len(sh), 2):
        bound = 1.0 / np.sqrt(sh[q][1])
        out.append(rng.uniform(-bound, bound, size=sh[q]).reshape(-1))
        out.append(rng.uniform(-bound, bound, size=sh[q + 1]).reshape(-1))
    return np.concatenate(out).astype(np.float32)


class Mlp:
    """One surrogate network on the handle's device."""

    def __init__(self, handle: Handle | None = None, n_in: int = NIN):
        self.h = handle or default_handle()
        self.lib = load_library()
        _declare(self.lib)
        p = C.c_void_p()
        self.h.check(self.lib.pcsdf_mlp_create(self.h.ptr, int(n_in),
                                               C.byref(p)))
        self.ptr = p
        self.n_in = int(n_in)
        self.nparam = nparam(self.n_in)
        self.in_offset = np.zeros(self.n_in, np.float32)
        self.in_scale = np.ones(self.n_in, np.float32)
        self.out_scale = 1.0

    def set_params(self, params, in_offset=None, in_scale=None,
                   out_scale=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.nparam:
            raise ValueError(f"need {self.nparam} parameters")
        if in_offset is not None:
            self.in_offset = np.ascontiguousarray(in_offset, np.float32)
        if in_scale is not None:
            self.in_scale = np.ascontiguousarray(in_scale, np.float32)
        if out_scale is not None:
            self.out_scale = float(out_scale)
        self.h.check(self.lib.pcsdf_mlp_set_params(
            self.ptr, p.ctypes.data_as(C.c_void_p),
            self.in_offset.ctypes.data_as(C.c_void_p),
            self.in_scale.ctypes.data_as(C.c_void_p), self.out_scale))

    def get_params(self) -> np.ndarray:
        p = np.empty(self.nparam, np.float32)
        self.h.check(self.lib.pcsdf_mlp_get_params(
            self.ptr, p.ctypes.data_as(C.c_void_p)))
        return p

    @staticmethod
    def _ptr(t):
        return None if t is None else C.c_void_p(t.data_ptr())

    @staticmethod
    def _stream(t):
        import torch
        return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)

    def forward(self, x, want_grad=True):
        """x: float32 [n, n_in] on the GPU -> (y [n], dy/dx [n, n_in] or
        None)."""
        import torch
        assert x.dtype == torch.float32 and x.is_contiguous() and \
            x.shape[-1] == self.n_in
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        g = torch.empty((n, self.n_in), dtype=torch.float32,
                        device=x.device) if want_grad else None
        self.h.check(self.lib.pcsdf_mlp_forward(
            self.ptr, n, self._ptr(x), self._ptr(y), self._ptr(g),
            self._stream(x)))
        return y, g

    def gradients(self, x, dy, want_grad_x=True):
        import torch
        n = x.shape[0]
        gp = torch.empty(self.nparam, dtype=torch.float32, device=x.device)
        gx = torch.empty((n, self.n_in), dtype=torch.float32,
                         device=x.device) if want_grad_x else None
        self.h.check(self.lib.pcsdf_mlp_gradients(
            self.ptr, n, self._ptr(x), self._ptr(dy), self._ptr(gp),
            self._ptr(gx), self._stream(x)))
        return gp, gx

    def train_step(self, x, target, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                   loss=None):
        n = x.shape[0]
        self.h.check(self.lib.pcsdf_mlp_train_step(
            self.ptr, n, self._ptr(x), self._ptr(target), float(lr),
            float(beta1), float(beta2), float(eps), self._ptr(loss),
            self._stream(x)))

    def loss_gradients(self, x, target, loss=None):
        """Gradient of the mean squared error w.r.t. every parameter
        (pcsdf_mlp_loss_gradients): float32 [nparam] on the GPU."""
        import torch
        n = x.shape[0]
        gp = torch.empty(self.nparam, dtype=torch.float32, device=x.device)
        self.h.check(self.lib.pcsdf_mlp_loss_gradients(
            self.ptr, n, self._ptr(x), self._ptr(target), self._ptr(gp),
            self._ptr(loss), self._stream(x)))
        return gp

    def adam_step(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step from a float32 [nparam] gradient on the GPU."""
        import torch
        assert grad.dtype == torch.float32 and grad.numel() == self.nparam
        self.h.check(self.lib.pcsdf_mlp_adam_step(
            self.ptr, self._ptr(grad), float(lr), float(beta1), float(beta2),
            float(eps), self._stream(grad)))

    def get_state(self):
        """(params, m1, m2, step): the optimiser's state, for checkpoints."""
        p, m1, m2 = (np.empty(self.nparam, np.float32) for _ in range(3))
        step = C.c_int64()
        self.h.check(self.lib.pcsdf_mlp_get_state(
            self.ptr, p.ctypes.data_as(C.c_void_p),
            m1.ctypes.data_as(C.c_void_p), m2.ctypes.data_as(C.c_void_p),
            C.byref(step)))
        return p, m1, m2, int(step.value)

    def set_state(self, params, m1, m2, step, in_offset, in_scale,
                  out_scale):
        """Restores what get_state returned, with the normalisation."""
        arrs = [np.ascontiguousarray(a, dtype=np.float32)
                for a in (params, m1, m2)]
        if any(a.size != self.nparam for a in arrs):
            raise ValueError(f"need {self.nparam} values per array")
        self.in_offset = np.ascontiguousarray(in_offset, np.float32)
        self.in_scale = np.ascontiguousarray(in_scale, np.float32)
        self.out_scale = float(out_scale)
        self.h.check(self.lib.pcsdf_mlp_set_state(
            self.ptr, *(a.ctypes.data_as(C.c_void_p) for a in arrs),
            int(step), self.in_offset.ctypes.data_as(C.c_void_p),
            self.in_scale.ctypes.data_as(C.c_void_p), self.out_scale))

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.pcsdf_mlp_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def surrogate_human_features(grid, human_xy, radius, height, centre,
                             slice_, human=None, label=None,
                             handle: Handle | None = None):
    """Rows of the per-human surrogate (pcsdf_surrogate_human_features):
    centre [n, 3] float32, slice_ [n] int32, human [n] int32 (None: 0) and
    label [n] float32 metres (None: no targets) on the GPU; human_xy host
    [n_slices, n_humans, 2].  Returns (x [n, 16], base d [n] voxels,
    target [n] voxels or None)."""
    import torch
    from . import _dev_ptr, _stream
    g = as_grid(grid)
    h = handle or default_handle()
    lib = load_library()
    _declare(lib)
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n = slice_.numel()
    dev = centre.device
    x = torch.empty((n, NIN), dtype=torch.float32, device=dev)
    base = torch.empty(n, dtype=torch.float32, device=dev)
    tgt = torch.empty(n, dtype=torch.float32, device=dev) \
        if label is not None else None
    h.check(lib.pcsdf_surrogate_human_features(
        h.ptr, C.byref(g), xy.shape[0], xy.shape[1],
        xy.ctypes.data_as(C.c_void_p), float(radius), float(height), n,
        _dev_ptr(centre, torch.float32, "centre", 3 * n),
        _dev_ptr(slice_, torch.int32, "slice", n),
        _dev_ptr(human, torch.int32, "human", n),
        _dev_ptr(label, torch.float32, "label", n),
        _dev_ptr(x, torch.float32, "x"), _dev_ptr(base, torch.float32, "base"),
        _dev_ptr(tgt, torch.float32, "target"), _stream(dev)))
    return x, base, tgt


def query_spheres_surrogate(net: Mlp, grid, static_ssq, static_sdf, human_xy,
                            radius, height, centre, sphere_radius, slice_,
                            fallback_margin=0.10, band=None, hinge_eps=0.0,
                            want_status=True, want_cost=False,
                            want_rows=False):
    """Sphere queries by the per-human network with exact fallback
    (pcsdf_query_spheres_surrogate).  band: metres (None: 2 sqrt(3) h, every
    cell where the nearest candidate may change).  Returns a dict with
    dist, grad, status, cost (or None), used_fallback and rows (the
    network's row count as a 1-element int32 tensor, or None)."""
    import torch
    from . import _dev_ptr, _stream
    g = as_grid(grid)
    h = net.h
    xy = np.ascontiguousarray(np.asarray(human_xy, dtype=np.float64))
    if xy.ndim != 3 or xy.shape[2] != 2:
        raise ValueError("human_xy must have shape [n_slices, n_humans, 2]")
    n_slices, K = xy.shape[0], xy.shape[1]
    if band is None:
        band = 2.0 * np.sqrt(3.0) * g.voxel_m
    V = g.nvox
    dev = centre.device
    n = slice_.numel()
    dist = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty((n, 3), dtype=torch.float32, device=dev)
    status = torch.empty(n, dtype=torch.uint8, device=dev) \
        if want_status else None
    cost = torch.empty(n, dtype=torch.float32, device=dev) \
        if want_cost else None
    used = torch.empty(n, dtype=torch.uint8, device=dev)
    rows = torch.zeros(1, dtype=torch.int32, device=dev) if want_rows \
        else None
    h.check(net.lib.pcsdf_query_spheres_surrogate(
        h.ptr, net.ptr, C.byref(g),
        _dev_ptr(static_ssq, torch.int32, "static_ssq", V),
        _dev_ptr(static_sdf, torch.float32, "static_sdf", V), n_slices, K,
        xy.ctypes.data_as(C.c_void_p) if K > 0 else None, float(radius),
        float(height), float(fallback_margin), float(band), n,
        _dev_ptr(centre, torch.float32, "centre", 3 * n),
        _dev_ptr(sphere_radius, torch.float32, "radius", n),
        _dev_ptr(slice_, torch.int32, "slice", n), float(hinge_eps),
        _dev_ptr(dist, torch.float32, "dist"),
        _dev_ptr(grad, torch.float32, "grad"),
        _dev_ptr(status, torch.uint8, "status"),
        _dev_ptr(cost, torch.float32, "cost"),
        _dev_ptr(used, torch.uint8, "used"),
        _dev_ptr(rows, torch.int32, "rows"), _stream(dev)))
    return {"dist": dist, "grad": grad, "status": status, "cost": cost,
            "used_fallback": used, "rows": rows}

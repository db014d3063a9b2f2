"""Binding of the surrogate MLP (pcsdf_mlp_*).

The network, its gradients and its optimiser step all run in the
library's HIP kernels; this module marshals torch tensors and host arrays.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from ._native import Handle, default_handle, load_library

NPARAM = 52609
NIN = 22
SHAPES = [(128, 22), (128,), (128, 128), (128,), (128, 128), (128,),
          (128, 128), (128,), (1, 128), (1,)]


def _declare(lib):
    if getattr(lib, "_mlp_declared", False):
        return
    P = C.c_void_p
    i32, f32 = C.c_int32, C.c_float
    lib.pcsdf_mlp_create.argtypes = [P, C.POINTER(P)]
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
    lib._mlp_declared = True


def init_params(rng: np.random.Generator) -> np.ndarray:
    """Uniform(+-1/sqrt(fan_in)) weights and biases (the numbers drawn on
    the host and passed to the library)."""
    out = []
    for q in range(0, len(SHAPES), 2):
        bound = 1.0 / np.sqrt(SHAPES[q][1])
        out.append(rng.uniform(-bound, bound, size=SHAPES[q]).reshape(-1))
        out.append(rng.uniform(-bound, bound, size=SHAPES[q + 1]).reshape(-1))
    return np.concatenate(out).astype(np.float32)


class Mlp:
    """One surrogate network on the handle's device."""

    def __init__(self, handle: Handle | None = None):
        self.h = handle or default_handle()
        self.lib = load_library()
        _declare(self.lib)
        p = C.c_void_p()
        self.h.check(self.lib.pcsdf_mlp_create(self.h.ptr, C.byref(p)))
        self.ptr = p
        self.in_offset = np.zeros(NIN, np.float32)
        self.in_scale = np.ones(NIN, np.float32)
        self.out_scale = 1.0

    def set_params(self, params, in_offset=None, in_scale=None,
                   out_scale=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != NPARAM:
            raise ValueError(f"need {NPARAM} parameters")
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
        p = np.empty(NPARAM, np.float32)
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
        """x: float32 [n, 22] on the GPU -> (y [n], dy/dx [n, 22] or None)."""
        import torch
        assert x.dtype == torch.float32 and x.is_contiguous() and \
            x.shape[-1] == NIN
        n = x.shape[0]
        y = torch.empty(n, dtype=torch.float32, device=x.device)
        g = torch.empty((n, NIN), dtype=torch.float32, device=x.device) \
            if want_grad else None
        self.h.check(self.lib.pcsdf_mlp_forward(
            self.ptr, n, self._ptr(x), self._ptr(y), self._ptr(g),
            self._stream(x)))
        return y, g

    def gradients(self, x, dy, want_grad_x=True):
        import torch
        n = x.shape[0]
        gp = torch.empty(NPARAM, dtype=torch.float32, device=x.device)
        gx = torch.empty((n, NIN), dtype=torch.float32, device=x.device) \
            if want_grad_x else None
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

    def close(self):
        if getattr(self, "ptr", None):
            self.lib.pcsdf_mlp_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

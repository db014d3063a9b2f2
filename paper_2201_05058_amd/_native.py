"""ctypes binding of libpcsdf.so (declared in include/pcsdf.h).

Argument marshalling only: every step of the path runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  If
the shared library is missing the import of the functions fails loudly;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpcsdf.so")

OK = 0
STATUS_NAMES = {
    0: "PCSDF_OK", 1: "PCSDF_ERR_INVALID_ARG", 2: "PCSDF_ERR_DIMS",
    3: "PCSDF_ERR_ALIGN", 4: "PCSDF_ERR_OOM", 5: "PCSDF_ERR_HIP",
    6: "PCSDF_ERR_NUMERIC",
}
Q_OOR_X, Q_OOR_Y, Q_OOR_Z = 1, 2, 4
Q_SLICE_CLAMPED, Q_INF_CORNER, Q_SLICE_NEG = 8, 16, 32
KERNEL_COMPOSITE, KERNEL_PLANES, KERNEL_QUERY, KERNEL_STATIC = 0, 1, 2, 3
KERNEL_BATCH, KERNEL_MLP, KERNEL_MLP_TRAIN, KERNEL_SURROGATE_DECIDE = 4, 5, 6, 7
KERNEL_RECOMPUTE, KERNEL_TEMPLATE, KERNEL_FACTORS = 8, 9, 10


class PcsdfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


class Grid(C.Structure):
    """pcsdf_grid: nx, ny, nz in [1, 1024], voxel size and origin (m)."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("reserved", C.c_int32), ("voxel_m", C.c_double),
                ("origin_m", C.c_double * 3)]

    @classmethod
    def make(cls, nx, ny, nz, voxel_m, origin=(0.0, 0.0, 0.0)):
        g = cls()
        g.nx, g.ny, g.nz, g.reserved = int(nx), int(ny), int(nz), 0
        g.voxel_m = float(voxel_m)
        for a in range(3):
            g.origin_m[a] = float(origin[a])
        return g

    @property
    def nvox(self):
        return self.nx * self.ny * self.nz

    @property
    def shape_zyx(self):
        return (self.nz, self.ny, self.nx)


class Scene(C.Structure):
    """pcsdf_scene: one scene of a batch."""
    _fields_ = [("grid", Grid), ("static_ssq_dev", C.c_void_p),
                ("n_slices", C.c_int32), ("n_humans", C.c_int32),
                ("human_xy_host", C.c_void_p), ("radius_m", C.c_double),
                ("height_m", C.c_double), ("out_ssq_dev", C.c_void_p),
                ("out_sdf_dev", C.c_void_p)]


class Tuning(C.Structure):
    """pcsdf_tuning: launch shapes (0 = library default)."""
    _fields_ = [("composite_slices_per_block", C.c_int32),
                ("batch_slices_per_item", C.c_int32),
                ("batch_chunk_quads", C.c_int32),
                ("batch_blocks_per_cu", C.c_int32),
                ("static_segments", C.c_int32),
                ("composite_order", C.c_int32),
                ("composite_static16", C.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

    @classmethod
    def from_dict(cls, d):
        t = cls()
        for f, _ in cls._fields_:
            setattr(t, f, int(d.get(f, 0)))
        return t


def as_grid(g) -> Grid:
    """A Grid from a Grid, or from any object with nx, ny, nz, h, origin."""
    if isinstance(g, Grid):
        return g
    return Grid.make(g.nx, g.ny, g.nz, g.h, getattr(g, "origin", (0, 0, 0)))


_lib = None
_lock = threading.Lock()


def load_library():
    """Loads libpcsdf.so and declares the C-ABI signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "`python -m paper_2201_05058_amd.build_lib` (hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        GP = C.POINTER(Grid)
        i32, f64 = C.c_int32, C.c_double
        lib.pcsdf_create.argtypes = [C.POINTER(P)]
        lib.pcsdf_create.restype = C.c_int
        lib.pcsdf_destroy.argtypes = [P]
        lib.pcsdf_destroy.restype = None
        lib.pcsdf_last_error.argtypes = [P]
        lib.pcsdf_last_error.restype = C.c_char_p
        lib.pcsdf_status_string.argtypes = [C.c_int]
        lib.pcsdf_status_string.restype = C.c_char_p
        lib.pcsdf_build_static_sdf.argtypes = [P, GP, P, P, P, P]
        lib.pcsdf_build_static_sdf.restype = C.c_int
        lib.pcsdf_predicted_composite_sdf.argtypes = [
            P, GP, P, i32, i32, P, f64, f64, P, P, P]
        lib.pcsdf_predicted_composite_sdf.restype = C.c_int
        lib.pcsdf_predicted_composite_sdf_noalloc.argtypes = [
            P, GP, P, i32, i32, P, f64, f64, P, P, P]
        lib.pcsdf_predicted_composite_sdf_noalloc.restype = C.c_int
        lib.pcsdf_predicted_composite_sdf_growing.argtypes = [
            P, GP, P, i32, i32, P, P, f64, P, P, P]
        lib.pcsdf_predicted_composite_sdf_growing.restype = C.c_int
        lib.pcsdf_recompute_sdf.argtypes = [
            P, GP, P, i32, i32, P, f64, f64, P, P, P]
        lib.pcsdf_recompute_sdf.restype = C.c_int
        lib.pcsdf_template_composite_sdf.argtypes = [
            P, GP, P, i32, i32, P, f64, f64, P, P, P]
        lib.pcsdf_template_composite_sdf.restype = C.c_int
        lib.pcsdf_obstacle_factors.argtypes = [
            P, GP, P, i32, i32, i32, P, P, P, f64, f64, P, P, P, P]
        lib.pcsdf_obstacle_factors.restype = C.c_int
        lib.pcsdf_build_floor_sdf.argtypes = [P, GP, P, i32, i32, P, P, P]
        lib.pcsdf_build_floor_sdf.restype = C.c_int
        lib.pcsdf_query_spheres_direct.argtypes = [
            P, GP, P, i32, i32, P, f64, f64, i32, P, P, P, f64, P, P, P, P, P]
        lib.pcsdf_query_spheres_direct.restype = C.c_int
        lib.pcsdf_query_spheres.argtypes = [
            P, GP, P, i32, i32, P, P, P, f64, P, P, P, P, P]
        lib.pcsdf_query_spheres.restype = C.c_int
        lib.pcsdf_profile_enable.argtypes = [P, C.c_int]
        lib.pcsdf_profile_enable.restype = C.c_int
        lib.pcsdf_profile_select.argtypes = [P, C.c_uint32]
        lib.pcsdf_profile_select.restype = C.c_int
        lib.pcsdf_profile_read.argtypes = [P, C.c_int,
                                           C.POINTER(C.c_double),
                                           C.POINTER(C.c_int64)]
        lib.pcsdf_profile_read.restype = C.c_int
        lib.pcsdf_profile_reset.argtypes = [P]
        lib.pcsdf_profile_reset.restype = C.c_int
        SP = C.POINTER(Scene)
        TP = C.POINTER(Tuning)
        lib.pcsdf_set_tuning.argtypes = [P, TP]
        lib.pcsdf_set_tuning.restype = C.c_int
        lib.pcsdf_get_tuning.argtypes = [P, TP]
        lib.pcsdf_get_tuning.restype = C.c_int
        lib.pcsdf_predicted_composite_sdf_batch.argtypes = [P, i32, SP, P]
        lib.pcsdf_predicted_composite_sdf_batch.restype = C.c_int
        lib.pcsdf_batch_graph_create.argtypes = [P, i32, SP, P,
                                                 C.POINTER(P)]
        lib.pcsdf_batch_graph_create.restype = C.c_int
        lib.pcsdf_batch_graph_set_positions.argtypes = [P, i32, P]
        lib.pcsdf_batch_graph_set_positions.restype = C.c_int
        lib.pcsdf_batch_graph_launch.argtypes = [P, P]
        lib.pcsdf_batch_graph_launch.restype = C.c_int
        lib.pcsdf_batch_graph_destroy.argtypes = [P]
        lib.pcsdf_batch_graph_destroy.restype = None
        lib.pcsdf_autotune_batch.argtypes = [P, i32, SP, P, i32, TP,
                                             C.POINTER(C.c_double)]
        lib.pcsdf_autotune_batch.restype = C.c_int
        lib.pcsdf_autotune_composite.argtypes = [P, SP, P, i32, TP,
                                                 C.POINTER(C.c_double)]
        lib.pcsdf_autotune_composite.restype = C.c_int
        _lib = lib
        return lib


class Handle:
    """Owns a pcsdf_handle (its workspace lives on the first device used)."""

    def __init__(self):
        self.lib = load_library()
        h = C.c_void_p()
        rc = self.lib.pcsdf_create(C.byref(h))
        if rc != OK:
            raise PcsdfError(rc, "pcsdf_create failed")
        self.ptr = h

    def check(self, rc: int):
        if rc != OK:
            msg = self.lib.pcsdf_last_error(self.ptr).decode()
            raise PcsdfError(rc, msg)

    # -- kernel timing with HIP events (PCSDF_KERNEL_* ids) --
    def profile(self, on: bool = True, only=None):
        """Kernel timing on or off; `only` lists the PCSDF_KERNEL_* ids to
        time (every id when None)."""
        if on and only is not None:
            mask = 0
            for k in only:
                mask |= 1 << int(k)
            self.check(self.lib.pcsdf_profile_select(self.ptr, mask))
        else:
            self.check(self.lib.pcsdf_profile_enable(self.ptr, int(bool(on))))

    def profile_reset(self):
        self.check(self.lib.pcsdf_profile_reset(self.ptr))

    def profile_read(self, kernel_id: int):
        """(total milliseconds, number of timed regions) of one id."""
        ms = C.c_double()
        n = C.c_int64()
        self.check(self.lib.pcsdf_profile_read(self.ptr, int(kernel_id),
                                               C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def set_tuning(self, t):
        if isinstance(t, dict):
            t = Tuning.from_dict(t)
        self.check(self.lib.pcsdf_set_tuning(self.ptr, C.byref(t)))

    def get_tuning(self) -> "Tuning":
        t = Tuning()
        self.check(self.lib.pcsdf_get_tuning(self.ptr, C.byref(t)))
        return t

    def close(self):
        if self.ptr:
            self.lib.pcsdf_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_tls = threading.local()


def default_handle() -> Handle:
    h = getattr(_tls, "handle", None)
    if h is None:
        h = Handle()
        _tls.handle = h
    return h

"""CPU oracle for the predicted composite distance field.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library
(``paper_2201_05058_amd``) never imports it and shares no code with it.

The arithmetic lives in ``pcsdf_oracle.c`` (plain C, built with gcc by
:func:`build` single-threaded, and once more with OpenMP for the CPU
baseline's all-core timing: ``omp=True`` on the calls that take it);
this module only marshals numpy arrays.  Every
function cites the passage of Finean et al. (2022) it restates in the C
source.  Parity status: every function here is pinned by the CPU tests in
``tests/test_oracle_pins.py`` (brute force, closed forms, invariants).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pcsdf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_libs = {}

INF32 = np.iinfo(np.int32).max
INF64 = np.iinfo(np.int64).max

OOR_X, OOR_Y, OOR_Z = 1, 2, 4
SLICE_CLAMPED, INF_CORNER, SLICE_NEG = 8, 16, 32


def _compile(out: str, omp: bool):
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall",
           "-fopenmp" if omp else "-Wno-unknown-pragmas", "-o", tmp, _SRC,
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA
    contraction) into ``oracle/liboracle.so`` (single-threaded) and
    ``oracle/liboracle_omp.so`` (the same source with OpenMP)."""
    for path, omp in ((_LIB, False), (_LIB_OMP, True)):
        if force or not os.path.exists(path) or \
                os.path.getmtime(path) < os.path.getmtime(_SRC):
            _compile(path, omp)
    _libs.clear()
    return _LIB


def threads(omp: bool = True) -> int:
    """Threads the OpenMP build's loops use (OMP_NUM_THREADS, else every
    core the process may run on); 1 for the plain build."""
    return int(_load(omp).or_threads())


def _load(omp: bool = False):
    key = bool(omp)
    if key in _libs:
        return _libs[key]
    path = _LIB_OMP if omp else _LIB
    if not os.path.exists(path) or \
            os.path.getmtime(path) < os.path.getmtime(_SRC):
        _compile(path, omp)
    lib = C.CDLL(path)
    P = C.c_void_p
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    lib.or_edt_sq.argtypes = [P, i32, i32, i32, P]
    lib.or_edt_sq.restype = C.c_int
    lib.or_edt_sq_order.argtypes = [P, i32, i32, i32, P, P]
    lib.or_edt_sq_order.restype = C.c_int
    lib.or_envelope_1d.argtypes = [P, i32, P]
    lib.or_envelope_1d.restype = C.c_int
    lib.or_signed_sq.argtypes = [P, i32, i32, i32, P]
    lib.or_signed_sq.restype = C.c_int
    lib.or_F.argtypes = [i32, f64]
    lib.or_F.restype = C.c_float
    lib.or_to_float.argtypes = [P, i64, f64, P]
    lib.or_to_float.restype = None
    lib.or_human_occupancy.argtypes = [i32, i32, i32, f64, f64, f64, f64,
                                       i32, P, f64, f64, P]
    lib.or_human_occupancy.restype = C.c_int
    lib.or_composite.argtypes = [P, P, i64, P]
    lib.or_composite.restype = None
    lib.or_build_static.argtypes = [P, i32, i32, i32, f64, P, P]
    lib.or_build_static.restype = C.c_int
    lib.or_predicted_composite.argtypes = [P, i32, i32, i32, f64, f64, f64,
                                           f64, i32, i32, P, f64, f64, P, P]
    lib.or_predicted_composite.restype = C.c_int
    lib.or_edt_at.argtypes = [P, i32, i32, i32, i32, i32, i32, i32]
    lib.or_edt_at.restype = i64
    lib.or_ssq_at.argtypes = [P, i32, i32, i32, i32, i32, i32]
    lib.or_ssq_at.restype = i32
    lib.or_query.argtypes = [P, i32, i32, i32, i32, f64, f64, f64, f64, i32,
                             P, P, P, f64, P, P, P, P]
    lib.or_query.restype = None
    lib.or_threads.argtypes = []
    lib.or_threads.restype = C.c_int
    _libs[key] = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def edt_sq(mask: np.ndarray) -> np.ndarray:
    """E_S (int64, INF64 where S is empty) of mask[z, y, x] != 0."""
    m = _u8(mask)
    nz, ny, nx = m.shape
    out = np.empty(m.shape, dtype=np.int64)
    if _load().or_edt_sq(_p(m), nx, ny, nz, _p(out)):
        raise MemoryError("oracle edt_sq")
    return out


def edt_sq_order(mask: np.ndarray, order) -> np.ndarray:
    """E_S with the three 1-D passes applied in `order` (axes 0=x,1=y,2=z)."""
    m = _u8(mask)
    nz, ny, nx = m.shape
    out = np.empty(m.shape, dtype=np.int64)
    o = np.asarray(order, dtype=np.int32)
    if _load().or_edt_sq_order(_p(m), nx, ny, nz, _p(o), _p(out)):
        raise MemoryError("oracle edt_sq_order")
    return out


def envelope_1d(f: np.ndarray) -> np.ndarray:
    """g(q) = min_p f(p) + (q-p)^2 with INF64 entries skipped."""
    f = np.ascontiguousarray(f, dtype=np.int64)
    out = np.empty_like(f)
    if _load().or_envelope_1d(_p(f), len(f), _p(out)):
        raise MemoryError("oracle envelope")
    return out


def signed_sq(mask: np.ndarray) -> np.ndarray:
    """SSQ_S: E_S outside S, -E_{G\\S} inside, int32 with +-INT32_MAX."""
    m = _u8(mask)
    nz, ny, nx = m.shape
    out = np.empty(m.shape, dtype=np.int32)
    if _load().or_signed_sq(_p(m), nx, ny, nz, _p(out)):
        raise MemoryError("oracle signed_sq")
    return out


def to_float(ssq: np.ndarray, h: float) -> np.ndarray:
    """F(x) = sign(x) * (float)h * sqrtf(|x|), +-inf for +-INT32_MAX."""
    x = np.ascontiguousarray(ssq, dtype=np.int32)
    out = np.empty(x.shape, dtype=np.float32)
    _load().or_to_float(_p(x), x.size, float(h), _p(out))
    return out


def human_occupancy(grid, xy: np.ndarray, radius: float,
                    height: float) -> np.ndarray:
    """Voxelised union of vertical cylinders for one slice; xy [K, 2]."""
    xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
    out = np.empty(grid.shape_zyx, dtype=np.uint8)
    ox, oy, oz = grid.origin
    rc = _load().or_human_occupancy(grid.nx, grid.ny, grid.nz, grid.h, ox,
                                    oy, oz, xy.shape[0], _p(xy), radius,
                                    height, _p(out))
    if rc:
        raise ValueError("oracle human_occupancy: non-finite or "
                         "out-of-range position")
    return out


def composite(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.int32)
    b = np.ascontiguousarray(b, dtype=np.int32)
    out = np.empty_like(a)
    _load().or_composite(_p(a), _p(b), a.size, _p(out))
    return out


def build_static(grid, occ: np.ndarray, omp: bool = False):
    """(SSQ_s int32, F(SSQ_s) fp32) of the static occupancy."""
    m = _u8(occ)
    ssq = np.empty(grid.shape_zyx, dtype=np.int32)
    sdf = np.empty(grid.shape_zyx, dtype=np.float32)
    if _load(omp).or_build_static(_p(m), grid.nx, grid.ny, grid.nz, grid.h,
                               _p(ssq), _p(sdf)):
        raise MemoryError("oracle build_static")
    return ssq, sdf


def predicted_composite(grid, static_ssq: np.ndarray, human_xy: np.ndarray,
                        radius: float, height: float, omp: bool = False):
    """Per-slice composite (int32 SSQ [n, nz, ny, nx], fp32 [n, ...])."""
    s = np.ascontiguousarray(static_ssq, dtype=np.int32)
    xy = np.ascontiguousarray(human_xy, dtype=np.float64)
    n, K = xy.shape[0], xy.shape[1]
    shp = (n,) + grid.shape_zyx
    ssq = np.empty(shp, dtype=np.int32)
    sdf = np.empty(shp, dtype=np.float32)
    ox, oy, oz = grid.origin
    rc = _load(omp).or_predicted_composite(_p(s), grid.nx, grid.ny, grid.nz,
                                        grid.h, ox, oy, oz, n, K, _p(xy),
                                        radius, height, _p(ssq), _p(sdf))
    if rc:
        raise ValueError("oracle predicted_composite failed")
    return ssq, sdf


def edt_at(mask: np.ndarray, want: int, i: int, j: int, k: int) -> int:
    """Brute force min over voxels u with (mask[u] != 0) == want of |v-u|^2."""
    m = _u8(mask)
    nz, ny, nx = m.shape
    return int(_load().or_edt_at(_p(m), int(bool(want)), nx, ny, nz, i, j, k))


def ssq_at(mask: np.ndarray, i: int, j: int, k: int) -> int:
    m = _u8(mask)
    nz, ny, nx = m.shape
    return int(_load().or_ssq_at(_p(m), nx, ny, nz, i, j, k))


def query(grid, sdf: np.ndarray, centre: np.ndarray, radius: np.ndarray,
          slices: np.ndarray, hinge_eps: float = 0.0):
    """Sphere queries: (dist f32 [Q], grad f32 [Q,3], status u8 [Q],
    cost f32 [Q])."""
    f = np.ascontiguousarray(sdf, dtype=np.float32)
    n_slices = f.shape[0] if f.ndim == 4 else 1
    c = np.ascontiguousarray(centre, dtype=np.float32).reshape(-1, 3)
    r = np.ascontiguousarray(radius, dtype=np.float32).reshape(-1)
    s = np.ascontiguousarray(slices, dtype=np.int32).reshape(-1)
    Q = c.shape[0]
    dist = np.empty(Q, dtype=np.float32)
    grad = np.empty((Q, 3), dtype=np.float32)
    st = np.empty(Q, dtype=np.uint8)
    cost = np.empty(Q, dtype=np.float32)
    ox, oy, oz = grid.origin
    _load().or_query(_p(f), n_slices, grid.nx, grid.ny, grid.nz, grid.h, ox,
                     oy, oz, Q, _p(c), _p(r), _p(s), float(hinge_eps),
                     _p(dist), _p(grad), _p(st), _p(cost))
    return dist, grad, st, cost

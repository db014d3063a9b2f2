"""C-ABI checks that need no GPU: the library loads, exports every entry
point its header declares, and rejects bad arguments on the host before
touching any device (fake device addresses are passed only to calls that
must fail validation)."""
import ctypes as C
import math
import os
import re

import pytest

import paper_2201_05058_amd as pc
from paper_2201_05058_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcsdf.h")

# Addresses never dereferenced: every call using them fails validation.
FAKE = C.c_void_p(0x10000)
FAKE_MIS = C.c_void_p(0x10002)


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pcsdf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("pcsdf_create", "pcsdf_destroy", "pcsdf_last_error",
              "pcsdf_build_static_sdf", "pcsdf_predicted_composite_sdf",
              "pcsdf_query_spheres"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_native.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings():
    lib = _native.load_library()
    assert lib.pcsdf_status_string(0) == b"PCSDF_OK"
    assert lib.pcsdf_status_string(6) == b"PCSDF_ERR_NUMERIC"
    assert lib.pcsdf_status_string(99) == b"PCSDF_ERR_UNKNOWN"


@pytest.fixture()
def h():
    hd = pc.Handle()
    yield hd
    hd.close()


def grid(nx=8, ny=8, nz=8, vox=0.05, origin=(0, 0, 0)):
    return _native.Grid.make(nx, ny, nz, vox, origin)


def comp(h, g, n=2, K=1, xy=None, r=0.25, H=1.8, static=FAKE, out=FAKE,
         outf=None):
    import numpy as np
    if xy is None:
        xy = np.zeros((n, K, 2))
    xy = np.ascontiguousarray(xy, dtype=np.float64)
    p = xy.ctypes.data_as(C.c_void_p) if xy.size else None
    return h.lib.pcsdf_predicted_composite_sdf(
        h.ptr, C.byref(g), static, n, K, p, r, H, out, outf, None)


def test_create_destroy_without_device():
    lib = _native.load_library()
    hp = C.c_void_p()
    assert lib.pcsdf_create(C.byref(hp)) == 0
    assert lib.pcsdf_last_error(hp) == b""
    lib.pcsdf_destroy(hp)
    lib.pcsdf_destroy(None)
    assert lib.pcsdf_create(None) == 1


@pytest.mark.parametrize("dims,code", [((0, 4, 4), 2), ((4, 1025, 4), 2),
                                       ((4, 4, -1), 2)])
def test_bad_dims(h, dims, code):
    g = grid(*dims)
    rc = h.lib.pcsdf_build_static_sdf(h.ptr, C.byref(g), FAKE, FAKE, None,
                                      None)
    assert rc == code
    assert "grid dimensions" in h.lib.pcsdf_last_error(h.ptr).decode()


def test_bad_voxel_and_origin(h):
    for vox in (0.0, -1.0, math.nan, math.inf):
        g = grid(vox=vox)
        assert h.lib.pcsdf_build_static_sdf(h.ptr, C.byref(g), FAKE, FAKE,
                                            None, None) == 6
    g = grid(origin=(0, math.nan, 0))
    assert h.lib.pcsdf_build_static_sdf(h.ptr, C.byref(g), FAKE, FAKE, None,
                                        None) == 6
    g = grid()
    g.reserved = 3
    assert h.lib.pcsdf_build_static_sdf(h.ptr, C.byref(g), FAKE, FAKE, None,
                                        None) == 1


def test_null_and_misaligned(h):
    g = grid()
    assert h.lib.pcsdf_build_static_sdf(h.ptr, C.byref(g), None, FAKE, None,
                                        None) == 1
    assert h.lib.pcsdf_build_static_sdf(h.ptr, C.byref(g), FAKE, FAKE_MIS,
                                        None, None) == 3
    assert h.lib.pcsdf_build_static_sdf(h.ptr, None, FAKE, FAKE, None,
                                        None) == 1
    assert comp(h, g, static=None) == 1
    assert comp(h, g, out=None, outf=None) == 1
    assert comp(h, g, out=FAKE_MIS) == 3


def test_composite_counts(h):
    import numpy as np
    g = grid()
    assert comp(h, g, n=0, xy=np.zeros((0, 1, 2))) == 1
    assert comp(h, g, K=300, xy=np.zeros((2, 300, 2))) == 1
    assert comp(h, g, K=-1, xy=np.zeros((0, 0, 2))) == 1
    rc = h.lib.pcsdf_predicted_composite_sdf(h.ptr, C.byref(g), FAKE, 2, 3,
                                             None, 0.25, 1.8, FAKE, None,
                                             None)
    assert rc == 1


def test_composite_numeric_inputs(h):
    import numpy as np
    g = grid()
    for bad in (math.nan, math.inf, -math.inf, 1e300):
        xy = np.zeros((3, 2, 2))
        xy[2, 1, 0] = bad
        assert comp(h, g, n=3, K=2, xy=xy) == 6
        assert "index 5" in h.lib.pcsdf_last_error(h.ptr).decode()
    for r, H in ((math.nan, 1.0), (0.25, math.inf), (-0.1, 1.0),
                 (0.25, -1.0), (1e6, 1.0)):
        assert comp(h, g, r=r, H=H) == 6


def test_query_validation(h):
    g = grid(nx=1)
    args = [FAKE, 1, 10, FAKE, FAKE, FAKE, 0.0, FAKE, FAKE, None, None, None]
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *args) == 2
    g = grid()
    a = list(args)
    a[1] = 0
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *a) == 1
    a = list(args)
    a[2] = -5
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *a) == 1
    a = list(args)
    a[6] = math.nan
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *a) == 6
    a = list(args)
    a[3] = None
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *a) == 1
    a = list(args)
    a[7] = FAKE_MIS
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *a) == 3
    # zero queries is a no-op that touches nothing
    a = list(args)
    a[2] = 0
    assert h.lib.pcsdf_query_spheres(h.ptr, C.byref(g), *a) == 0


def test_profile_calls_without_device(h):
    h.profile(True)
    ms, n = h.profile_read(_native.KERNEL_COMPOSITE)
    assert ms == 0.0 and n == 0
    h.profile_reset()
    with pytest.raises(pc.PcsdfError):
        h.profile_read(17)
    h.profile(True, only=[_native.KERNEL_COMPOSITE, _native.KERNEL_QUERY])
    assert h.lib.pcsdf_profile_select(h.ptr, 1 << 11) == 1  # beyond COUNT
    assert h.lib.pcsdf_profile_select(h.ptr, (1 << 11) - 1) == 0
    h.profile(False)


def test_surrogate_validation(h):
    """The surrogate's entry points reject bad arguments on the host."""
    import numpy as np
    from paper_2201_05058_amd import surrogate as sg
    sg._declare(h.lib)
    g = grid()
    xy = np.zeros((2, 1, 2))
    P = xy.ctypes.data_as(C.c_void_p)
    # no network
    assert h.lib.pcsdf_query_spheres_surrogate(
        h.ptr, None, C.byref(g), FAKE, FAKE, 2, 1, P, 0.25, 1.8, 0.1, 0.05,
        10, FAKE, FAKE, FAKE, 0.0, FAKE, FAKE, None, None, None, None,
        None) == 1

    def feat(n=5, n_humans=1, centre=FAKE, slices=FAKE, x=FAKE, label=None,
             target=None):
        return h.lib.pcsdf_surrogate_human_features(
            h.ptr, C.byref(g), 2, n_humans, P, 0.25, 1.8, n, centre, slices,
            None, label, x, None, target, None)
    assert feat(n=-1) == 1
    assert feat(n_humans=0) == 1
    assert feat(target=FAKE) == 1  # a target needs labels
    assert feat(centre=None) == 1
    assert feat(x=FAKE_MIS) == 3
    assert feat(n=0) == 0  # no work, nothing touched
    # the network's width: 1..32 inputs
    assert h.lib.pcsdf_mlp_param_count(16) == sg.nparam(16) == 51841
    assert h.lib.pcsdf_mlp_param_count(22) == 52609
    assert h.lib.pcsdf_mlp_param_count(0) == -1
    assert h.lib.pcsdf_mlp_param_count(33) == -1
    out = C.c_void_p()
    assert h.lib.pcsdf_mlp_create(h.ptr, 0, C.byref(out)) == 1
    assert h.lib.pcsdf_mlp_create(h.ptr, 33, C.byref(out)) == 1


def test_tuning_validation_without_device(h):
    """Launch shapes are checked on the host: negative values, more than 32
    workgroups per CU, chunk sizes off the 256-quad step, segment counts
    other than 0, 1, 2, 4 or 8, block orders other than 0 or 1 and static
    copy choices other than 0, 1 or 2 are rejected; accepted values read
    back unchanged."""
    from paper_2201_05058_amd._native import Tuning
    good = {"composite_slices_per_block": 3, "batch_slices_per_item": 2,
            "batch_chunk_quads": 512, "batch_blocks_per_cu": 8,
            "static_segments": 4, "composite_order": 1,
            "composite_static16": 2}
    h.set_tuning(good)
    assert h.get_tuning().as_dict() == good
    for bad in ({"composite_slices_per_block": -1}, {"batch_blocks_per_cu": 33},
                {"batch_chunk_quads": 100}, {"static_segments": 3},
                {"static_segments": 16}, {"static_segments": -2},
                {"composite_order": 2}, {"composite_order": -1},
                {"composite_static16": 3}, {"composite_static16": -1}):
        t = Tuning.from_dict(bad)
        assert h.lib.pcsdf_set_tuning(h.ptr, C.byref(t)) == 1, bad
    assert h.get_tuning().as_dict() == good  # rejected calls change nothing


def test_noalloc_composite_rejects_on_the_host(h):
    """The no-allocation composite refuses centre sets beyond its kernel
    arguments and planes beyond its scratch before touching a device."""
    import numpy as np
    f = h.lib.pcsdf_predicted_composite_sdf_noalloc
    g = grid(40, 40, 20)
    xy = np.zeros((50, 8, 2))
    rc = f(h.ptr, C.byref(g), FAKE, 50, 8, xy.ctypes.data_as(C.c_void_p),
           0.25, 1.8, FAKE, None, None)
    assert rc == 1 and b"exceeds 240" in h.lib.pcsdf_last_error(h.ptr)
    g = grid(1024, 1024, 2)
    xy = np.zeros((20, 1, 2))
    rc = f(h.ptr, C.byref(g), FAKE, 20, 1, xy.ctypes.data_as(C.c_void_p),
           0.25, 1.8, FAKE, None, None)
    assert rc == 1 and b"scratch" in h.lib.pcsdf_last_error(h.ptr)
    rc = f(h.ptr, C.byref(grid()), FAKE_MIS, 2, 1,
           xy.ctypes.data_as(C.c_void_p), 0.25, 1.8, FAKE, None, None)
    assert rc == 3

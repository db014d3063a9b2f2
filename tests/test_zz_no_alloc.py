"""The composite entry point that allocates nothing
(pcsdf_predicted_composite_sdf_noalloc), called through the C-ABI, against
pcsdf_predicted_composite_sdf: identical int32 and fp32 fields on calls in
a row, each with a smaller grid, fewer slices and humans (the shared
scratch keeps the previous call's contents), and the oracle on the first
and the last.  The first call's stack of planes (16 slices of 1024 x 128)
is large enough for the planar fields' separable path (coverage, row pass
and column pass), the others take the per-pixel kernel."""
import ctypes as C
import sys

import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def noalloc(pc, h, sc, ssq_s, dev):
    from paper_2201_05058_amd import _native
    g = _native.as_grid(sc.grid)
    n, K = sc.human_xy.shape[:2]
    shp = (n,) + sc.grid.shape_zyx
    oc = torch.full(shp, 7, dtype=torch.int32, device=dev)
    of = torch.full(shp, 7.0, dtype=torch.float32, device=dev)
    xy = np.ascontiguousarray(sc.human_xy, np.float64)
    torch.cuda.synchronize()
    rc = h.lib.pcsdf_predicted_composite_sdf_noalloc(
        h.ptr, C.byref(g), C.c_void_p(ssq_s.data_ptr()), n, K,
        xy.ctypes.data_as(C.c_void_p) if K else None, float(sc.radius),
        float(sc.height), C.c_void_p(oc.data_ptr()),
        C.c_void_p(of.data_ptr()),
        C.c_void_p(torch.cuda.current_stream(dev).cuda_stream))
    assert rc == 0, h.lib.pcsdf_last_error(h.ptr)
    torch.cuda.synchronize()
    return oc.cpu().numpy(), of.cpu().numpy()


def test_noalloc_matches_composite_twice(dev):
    import paper_2201_05058_amd as pc
    h = pc.Handle()
    scenes = [scenegen.small_scene(30, 1024, 128, 6, h=0.02, n_boxes=12,
                                   n_humans=4, n_slices=16),
              scenegen.small_scene(31, 96, 80, 40, h=0.04, n_boxes=8,
                                   n_humans=3, n_slices=6),
              scenegen.small_scene(32, 37, 29, 23, h=0.05, n_boxes=4,
                                   n_humans=2, n_slices=3)]
    for q, sc in enumerate(scenes):
        say(f"no-alloc composite call {q}: grid {sc.grid.shape_zyx} "
            f"slices {sc.n_slices} humans {sc.n_humans}")
        occ = torch.from_numpy(sc.occ).to(dev)
        ssq_s, _ = pc.build_static_sdf(sc.grid, occ, want_sdf=False,
                                       handle=h)
        c, cf = noalloc(pc, h, sc, ssq_s, dev)
        wc, wf = pc.predicted_composite_sdf(sc.grid, ssq_s, sc.human_xy,
                                            sc.radius, sc.height, handle=h)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(c, wc.cpu().numpy())
        np.testing.assert_array_equal(cf.view(np.int32),
                                      wf.cpu().numpy().view(np.int32))
        if q in (0, len(scenes) - 1):
            say("  against the oracle")
            rs, _ = oracle.build_static(sc.grid, sc.occ)
            oc, of = oracle.predicted_composite(sc.grid, rs, sc.human_xy,
                                                sc.radius, sc.height)
            np.testing.assert_array_equal(c, oc)
            np.testing.assert_array_equal(cf.view(np.int32),
                                          of.view(np.int32))
    h.close()


def test_noalloc_rejects_sizes_beyond_its_scratch(dev):
    import paper_2201_05058_amd as pc
    h = pc.Handle()
    sc = scenegen.small_scene(33, 40, 40, 20, h=0.05, n_humans=8,
                              n_slices=50)
    occ = torch.from_numpy(sc.occ).to(dev)
    ssq_s, _ = pc.build_static_sdf(sc.grid, occ, want_sdf=False, handle=h)
    with pytest.raises(Exception, match="exceeds 240"):
        pc.predicted_composite_sdf_noalloc(
            sc.grid, ssq_s, sc.human_xy, sc.radius, sc.height,
            torch.empty((50,) + sc.grid.shape_zyx, dtype=torch.int32,
                        device=dev), None, handle=h)
    h.close()


def test_noalloc_rejects_planes_beyond_its_scratch(dev):
    import paper_2201_05058_amd as pc
    from paper_2201_05058_amd import _native
    h = pc.Handle()
    g = _native.Grid.make(1024, 1024, 2, 0.01, (0, 0, 0))
    ssq_s = torch.full((2, 1024, 1024), 2 ** 31 - 1, dtype=torch.int32,
                       device=dev)
    xy = np.full((20, 1, 2), 5.0)
    with pytest.raises(Exception, match="scratch"):
        pc.predicted_composite_sdf_noalloc(
            g, ssq_s, xy, 0.25, 1.8, None,
            torch.empty((20, 2, 1024, 1024), dtype=torch.float32,
                        device=dev), handle=h)
    h.close()

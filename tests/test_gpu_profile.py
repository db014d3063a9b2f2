"""The library's kernel timing: regions selected by mask are the only ones
timed, a region counts calls (not kernels), and timing does not change
any output."""
import sys

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_profile_selection_and_counts(dev):
    import paper_2201_05058_amd as pc
    from paper_2201_05058_amd import _native
    sc = scenegen.small_scene(91, 40, 33, 20, h=0.05, n_humans=3,
                              n_slices=4)
    g = sc.grid
    h = pc.Handle()
    occ = torch.from_numpy(sc.occ).to(dev)
    ssq_s, _ = pc.build_static_sdf(g, occ, handle=h)

    def call():
        return pc.predicted_composite_sdf(g, ssq_s, sc.human_xy, sc.radius,
                                          sc.height, handle=h)

    ref_c, ref_f = call()
    torch.cuda.synchronize()
    say("profile: composite only")
    h.profile(True, only=[_native.KERNEL_COMPOSITE])
    h.profile_reset()
    outs = [call() for _ in range(3)]
    torch.cuda.synchronize()
    ms, n = h.profile_read(_native.KERNEL_COMPOSITE)
    assert n == 3 and ms > 0.0
    assert h.profile_read(_native.KERNEL_PLANES) == (0.0, 0)
    say("profile: every region")
    h.profile(True)
    h.profile_reset()
    outs += [call() for _ in range(2)]
    torch.cuda.synchronize()
    # three planar kernels per call, counted once per call
    ms_p, n_p = h.profile_read(_native.KERNEL_PLANES)
    assert n_p == 2 and ms_p > 0.0
    assert h.profile_read(_native.KERNEL_COMPOSITE)[1] == 2
    h.profile(False)
    h.profile_reset()
    call()
    torch.cuda.synchronize()
    assert h.profile_read(_native.KERNEL_COMPOSITE) == (0.0, 0)
    for c, f in outs:
        assert torch.equal(c, ref_c)
        assert torch.equal(f.view(torch.int32), ref_f.view(torch.int32))
    h.close()

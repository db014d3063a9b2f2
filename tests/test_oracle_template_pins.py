"""Pins of the compute-once-and-shift composite's oracle: with whole-voxel
motion, separate humans and cylinders inside the grid it must equal the
exact per-slice composite (the two definitions then coincide); at the
first slice a lone human inside the grid always gives the exact field; and
in general it differs from the exact field by at most the sub-voxel shift
and re-voxelisation (bounded here in metres)."""
import numpy as np
import pytest

import oracle
import scenegen
from oracle.template import template_composite


def _room(seed, nx=30, ny=26, nz=12, h=0.05):
    sc = scenegen.small_scene(seed, nx, ny, nz, h=h, n_boxes=3, n_humans=2,
                              n_slices=4)
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    return sc, rs


def test_whole_voxel_motion_equals_exact_composite():
    sc, rs = _room(81)
    h = sc.grid.h
    # two humans well inside the grid, apart, moving whole voxels per slice
    start = np.array([[8.3 * h, 9.6 * h], [21.1 * h, 16.4 * h]])
    step = np.array([[1, 0], [-1, 2]]) * h
    xy = start[None] + np.arange(4)[:, None, None] * step[None]
    r = 0.12
    got, gf = template_composite(sc.grid, rs, xy, r, 0.3)
    want, wf = oracle.predicted_composite(sc.grid, rs, xy, r, 0.3)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(gf, wf)


def test_first_slice_lone_human_is_exact():
    sc, rs = _room(82)
    xy = np.array([[[0.71, 0.63]], [[0.9, 0.8]]])
    got, _ = template_composite(sc.grid, rs, xy, 0.2, 1.8)
    want, _ = oracle.predicted_composite(sc.grid, rs, xy[:1], 0.2, 1.8)
    np.testing.assert_array_equal(got[0], want[0])


def test_subvoxel_motion_close_to_exact():
    # humans inside the grid moving by fractions of a voxel (a template is
    # unclipped, so a human straddling the grid's edge would differ more)
    sc, rs = _room(83)
    h = sc.grid.h
    start = np.array([[8.3 * h, 9.6 * h], [20.1 * h, 15.4 * h]])
    step = np.array([[0.37, -0.52], [-0.81, 0.66]]) * h
    xy = start[None] + np.arange(4)[:, None, None] * step[None]
    got, gf = template_composite(sc.grid, rs, xy, 0.14, sc.height)
    want, wf = oracle.predicted_composite(sc.grid, rs, xy, 0.14, sc.height)
    assert (got != want).any()
    free = (got > 0) & (want > 0) & np.isfinite(gf) & np.isfinite(wf)
    # a half-voxel shift per axis plus one voxel of re-voxelisation
    assert np.abs(gf[free] - wf[free]).max() <= 2.0 * sc.grid.h
    assert ((got < 0) == (want < 0)).mean() > 0.99


# Worked example of the shift rule (the nearest whole-voxel displacement,
# ties upward): a displacement of delta voxels moves the template by
#   +0.5 -> 1,  -0.5 -> 0,  -0.51 -> -1,  +1.49 -> 1   voxels.
# Truncation gives (0, 0, 0, 1), plain floor (0, -1, -1, 1), rounding
# half away from zero (1, -1, -1, 1) and half to even (0, 0, -1, 1): each
# differs from the rule in one case at least.  With h a power of two the
# fixed-point displacements are exact (32768, -32768, -33423, 97648 in
# units of 2^-16 voxel), and a lone human inside the grid shifted by d
# whole voxels has exactly the exact field of the human at x0 + d h.
@pytest.mark.parametrize("delta,d", [(0.5, 1), (-0.5, 0), (-0.51, -1),
                                     (1.49, 1)])
@pytest.mark.parametrize("axis", [0, 1])
def test_shift_rule_worked_example(delta, d, axis):
    h = 0.0625
    sc, rs = _room(84, nx=28, ny=24, nz=6, h=h)
    x0 = np.array([12.5 * h, 11.5 * h])  # a voxel centre
    x1 = x0.copy()
    x1[axis] += delta * h
    xy = np.stack([x0, x1])[:, None, :]
    got, _ = template_composite(sc.grid, rs, xy, 0.2, 0.25)
    whole = x0.copy()
    whole[axis] += d * h
    want, _ = oracle.predicted_composite(sc.grid, rs, whole[None, None, :],
                                         0.2, 0.25)
    np.testing.assert_array_equal(got[1], want[0])
    # the neighbouring whole shifts give other fields, so the check tells
    for other in (d - 1, d + 1):
        alt = x0.copy()
        alt[axis] += other * h
        wa, _ = oracle.predicted_composite(sc.grid, rs, alt[None, None, :],
                                           0.2, 0.25)
        assert (got[1] != wa[0]).any()

"""The oracle's OpenMP build (used only to time the CPU baseline on all
cores) against its plain single-threaded build: the same static fields and
composites, bit for bit, on ragged grids, empty and full maps and humans
partly outside the grid.  CPU only."""
import numpy as np
import pytest

import oracle
import scenegen


def cases():
    yield scenegen.small_scene(1, 67, 45, 29, h=0.05, n_boxes=6, n_humans=3,
                               n_slices=4)
    yield scenegen.small_scene(2, 1, 40, 33, h=0.05, n_boxes=3, n_humans=2,
                               n_slices=2)
    yield scenegen.small_scene(3, 90, 2, 7, h=0.05, n_boxes=4, n_humans=1,
                               n_slices=3)
    sc = scenegen.small_scene(4, 33, 31, 17, h=0.05, n_boxes=0, n_humans=2,
                              n_slices=2)
    sc.occ[:] = 0
    yield sc
    sc = scenegen.small_scene(5, 33, 31, 17, h=0.05, n_boxes=0, n_humans=2,
                              n_slices=2)
    sc.occ[:] = 1
    yield sc
    yield scenegen.cube64()


@pytest.mark.parametrize("idx", range(6))
def test_openmp_build_is_bit_identical(idx):
    assert oracle.threads(omp=False) == 1
    sc = list(cases())[idx]
    g = sc.grid
    a_ssq, a_sdf = oracle.build_static(g, sc.occ)
    b_ssq, b_sdf = oracle.build_static(g, sc.occ, omp=True)
    np.testing.assert_array_equal(a_ssq, b_ssq)
    np.testing.assert_array_equal(a_sdf.view(np.int32), b_sdf.view(np.int32))
    ac, af = oracle.predicted_composite(g, a_ssq, sc.human_xy, sc.radius,
                                        sc.height)
    bc, bf = oracle.predicted_composite(g, a_ssq, sc.human_xy, sc.radius,
                                        sc.height, omp=True)
    np.testing.assert_array_equal(ac, bc)
    np.testing.assert_array_equal(af.view(np.int32), bf.view(np.int32))

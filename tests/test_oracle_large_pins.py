"""The oracle's composite at the two large workloads against closed forms
at sampled voxels (boxes and voxelised cylinders; see closed_forms.py):
the 256x256x128 room (slices 0 and 19) and the 512x512x256 room with 8
humans on piecewise-linear paths (slice 0)."""
import numpy as np
import pytest

import oracle
import scenegen
from closed_forms import SampledClosedForm


@pytest.mark.parametrize("maker,slices", [("room256", (0, 19)),
                                          ("room512", (0,))])
def test_oracle_composite_matches_closed_forms(maker, slices):
    if maker == "room256":
        sc = scenegen.room256(n_queries=0)
    else:
        sc = scenegen.room512(with_queries=False)
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    chk = SampledClosedForm(sc, M=60_000, seed=1)
    ssq_s = chk.gather(rs)
    for j in slices:
        c, _ = oracle.predicted_composite(sc.grid, rs, sc.human_xy[j:j + 1],
                                          sc.radius, sc.height)
        free, inside = chk.check_slice(j, chk.gather(c[0]), ssq_s)
        assert free > 30_000  # most samples are outside every obstacle

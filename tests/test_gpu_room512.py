"""Parity at the largest workload: a 512x512x256 grid at 0.01 m (67M
voxels), 200 boxes, 8 humans on piecewise-linear paths, 50 slices at
0.05 s, 100k spheres per slice -- in the launch configuration the library
uses for it (one plain call for all 50 slices).

The oracle runs the full static field and three whole slices (first,
middle, last: about 7 s each on one core).  Every other slice is checked at
sampled voxels against closed forms that hold at any size: outside every
obstacle the composite is the squared distance to the union of the
environment's index boxes and the humans' voxelised cylinders, each a
minimum over boxes / over disk rows of clamped coordinate differences
(chords from the exact fixed-point predicate, computed here with Python
integers); inside the environment and outside the humans it is the static
field; inside a human it is negative.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from closed_forms import SampledClosedForm

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CHECK_SLICES = (0, 17, 49)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def run(dev):
    import paper_2201_05058_amd as pc
    sc = scenegen.room512(queries_per_slice=100_000)
    say("room512: gpu static + composite, 50 slices")
    occ = torch.from_numpy(sc.occ).to(dev)
    ssq_s, sdf_s = pc.build_static_sdf(sc.grid, occ)
    c, cf = pc.predicted_composite_sdf(sc.grid, ssq_s, sc.human_xy, sc.radius,
                                       sc.height)
    q = sc.queries
    d, g, st, _ = pc.query_spheres(sc.grid, cf, torch.from_numpy(q.centre).to(dev),
                                   torch.from_numpy(q.radius).to(dev),
                                   torch.from_numpy(q.slice).to(dev))
    torch.cuda.synchronize()
    out = {"sc": sc, "ssq_s": ssq_s, "sdf_s": sdf_s, "c": c, "cf": cf,
           "d": d.cpu().numpy(), "g": g.cpu().numpy(), "st": st.cpu().numpy()}
    yield out
    del out
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def static_oracle(run):
    sc = run["sc"]
    return oracle.build_static(sc.grid, sc.occ)


def test_static_full(run, static_oracle):
    rs, rf = static_oracle
    say("room512: static parity (67M voxels)")
    np.testing.assert_array_equal(run["ssq_s"].cpu().numpy(), rs)
    np.testing.assert_array_equal(run["sdf_s"].cpu().numpy(), rf)


@pytest.fixture(scope="module")
def slice_oracle(run, static_oracle):
    sc = run["sc"]
    rs, _ = static_oracle
    return {j: oracle.predicted_composite(sc.grid, rs, sc.human_xy[j:j + 1],
                                          sc.radius, sc.height)
            for j in CHECK_SLICES}


@pytest.mark.parametrize("j", CHECK_SLICES)
def test_slice_full(run, slice_oracle, j):
    say(f"room512: slice {j} vs oracle")
    wc, wf = slice_oracle[j]
    np.testing.assert_array_equal(run["c"][j].cpu().numpy(), wc[0])
    np.testing.assert_array_equal(run["cf"][j].cpu().numpy(), wf[0])


def test_all_slices_sampled_closed_form(run):
    sc = run["sc"]
    checker = SampledClosedForm(sc, M=40_000, seed=512)
    ssq_s = checker.gather(run["ssq_s"])
    say("room512: sampled closed-form check of all 50 slices")
    for j in range(sc.n_slices):
        checker.check_slice(j, checker.gather(run["c"][j]), ssq_s)


def test_queries_on_oracle_slices(run, slice_oracle):
    sc = run["sc"]
    q = sc.queries
    sel = np.isin(q.slice, CHECK_SLICES)
    say(f"room512: {int(sel.sum())} queries vs oracle")
    # the oracle query reads only the slices it is given: renumber them
    wfs = np.stack([slice_oracle[j][1][0] for j in CHECK_SLICES])
    remap = {s: t for t, s in enumerate(CHECK_SLICES)}
    sl = np.array([remap[s] for s in q.slice[sel]], np.int32)
    wd, wg, wst, _ = oracle.query(sc.grid, wfs, q.centre[sel], q.radius[sel],
                                  sl)
    d, g, st = run["d"][sel], run["g"][sel], run["st"][sel]
    np.testing.assert_array_equal(st, wst)
    err = np.abs(d.astype(np.float64) - wd)
    assert (err <= 1e-6 * np.maximum(np.abs(wd), sc.grid.h)).all()
    err = np.abs(g.astype(np.float64) - wg)
    assert (err <= 1e-6 * np.maximum(np.abs(wg), 1.0)).all()


@pytest.mark.parametrize("G,order,copy", [(5, 0, 0), (10, 0, 0), (25, 0, 0),
                                          (2, 1, 0), (2, 0, 1)])
def test_other_slice_groups_give_identical_bytes(run, G, order, copy):
    """The composite in other launch shapes the autotuner may pick for
    this workload (slice groups of 5, 10 and 25 per block row; the XCD
    block order) and without the 16-bit static copy: the same bytes as the
    default shape checked above, for all 50 slices."""
    import paper_2201_05058_amd as pc
    sc = run["sc"]
    say(f"room512: composite with {G} slices per block row, order {order}, "
        f"static16 {copy}")
    h = pc.Handle()
    try:
        h.set_tuning({"composite_slices_per_block": G,
                      "composite_order": order,
                      "composite_static16": copy})
        c, cf = pc.predicted_composite_sdf(sc.grid, run["ssq_s"], sc.human_xy,
                                           sc.radius, sc.height, handle=h)
        torch.cuda.synchronize()
        assert torch.equal(c, run["c"])
        assert torch.equal(cf.view(torch.int32), run["cf"].view(torch.int32))
        del c, cf
    finally:
        h.close()
    torch.cuda.empty_cache()


def test_surrogate_queries_on_oracle_slices(run, slice_oracle,
                                            static_oracle):
    """The trained room512 surrogate (eight humans on piecewise-linear
    paths) on the workload's spheres of slices 0, 17 and 49, against the
    oracle's rule given the GPU network's values for every (query, human)
    row and the oracle's exact fields of those slices for the fallback:
    identical decisions, bit-identical answered distances, gradients
    within 1e-6, fallback answers within the exact-query contract."""
    import os

    from oracle import surrogate as osur
    from paper_2201_05058_amd import surrogate as sg
    from paper_2201_05058_amd import train
    sc = run["sc"]
    dev = run["ssq_s"].device
    w = os.path.join(os.path.dirname(__file__), "..", "paper_2201_05058_amd",
                     "weights", "surrogate_room512.npz")
    net, _ = train.load(w)
    q = sc.queries
    sel = np.nonzero(np.isin(q.slice, CHECK_SLICES))[0][::10]
    c, r, s = q.centre[sel], q.radius[sel], q.slice[sel]
    say(f"room512: {len(sel)} surrogate queries vs oracle")
    td = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = sg.query_spheres_surrogate(
        net, sc.grid, run["ssq_s"], run["sdf_s"], sc.human_xy, sc.radius,
        sc.height, td(c), td(r), td(s), want_cost=True)
    torch.cuda.synchronize()
    # the oracle on the three slices (queries renumbered 0, 1, 2)
    remap = {j: t for t, j in enumerate(CHECK_SLICES)}
    s3 = np.array([remap[int(j)] for j in s], np.int32)
    xy3 = sc.human_xy[list(CHECK_SLICES)]
    wf3 = np.concatenate([slice_oracle[j][1] for j in CHECK_SLICES])
    rows = {}

    def gpu_net(x, k):
        if k not in rows:
            kk = np.full(len(s), k, np.int32)
            xd, _, _ = sg.surrogate_human_features(
                sc.grid, sc.human_xy, sc.radius, sc.height, td(c), td(s),
                human=td(kk))
            y, gx = net.forward(xd)
            torch.cuda.synchronize()
            rows[k] = (y.cpu().numpy(), gx.cpu().numpy())
        return rows[k]
    _, rf = static_oracle
    wd, wg, wst, wcost, wused = osur.query(
        sc.grid, wf3, rf, gpu_net, xy3, sc.radius, sc.height, c, r, s3,
        margin=0.10, band=2 * np.sqrt(3) * sc.grid.h)
    d = out["dist"].cpu().numpy()
    gr = out["grad"].cpu().numpy()
    used = out["used_fallback"].cpu().numpy()
    np.testing.assert_array_equal(used, wused)
    acc = used == 0
    say(f"  answered {acc.mean():.3f}")
    assert acc.mean() > 0.1
    np.testing.assert_array_equal(d[acc], wd[acc])
    np.testing.assert_array_equal(out["status"].cpu().numpy(), wst)
    assert np.all(np.abs(gr[acc] - wg[acc]) <=
                  1e-6 * np.maximum(np.abs(wg[acc]), 1.0))
    ex = ~acc
    assert np.all(np.abs(d[ex] - wd[ex]) <=
                  1e-6 * np.maximum(np.abs(wd[ex]), sc.grid.h))
    net.close()

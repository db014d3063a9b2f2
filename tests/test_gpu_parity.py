"""Parity of the HIP path (through the C-ABI) with the CPU oracle.

Squared distances must be bit-exact; fp32 fields and query outputs within
1e-6 relative (with the floors of the query contract).  Inputs are seeded
synthetic scenes; expected values come only from the oracle.
"""
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


@pytest.fixture(scope="module")
def pc(dev):
    import paper_2201_05058_amd as m
    m.load_library()
    return m


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def assert_f32_close(got, want, rel=1e-6):
    got = np.asarray(got)
    want = np.asarray(want)
    fin = np.isfinite(want)
    assert (np.isfinite(got) == fin).all()
    np.testing.assert_array_equal(got[~fin], want[~fin])
    err = np.abs(got[fin].astype(np.float64) - want[fin].astype(np.float64))
    assert (err <= rel * np.abs(want[fin].astype(np.float64))).all(), \
        float(err.max())


def gpu_static(pc, grid, occ, dev):
    occ_d = to_dev(occ.astype(np.uint8), dev)
    ssq, sdf = pc.build_static_sdf(grid, occ_d)
    torch.cuda.synchronize()
    return ssq, sdf


# ------------------------------------------------------------ static build

# Passes with fewer than 64 column tiles of 32 run one lane per voxel (a
# search outward along the column), the others the segmented envelopes:
# the small and one-layer shapes take the first, the larger the second.
STATIC_SHAPES = [  # (nz, ny, nx)
    (1, 1, 1), (1, 1, 9), (1, 7, 1), (5, 1, 1), (4, 5, 6), (12, 12, 12),
    (29, 131, 67), (33, 70, 130), (3, 2, 200), (7, 64, 64), (2, 3, 1024),
    (1, 300, 257), (1, 256, 256), (5, 9, 264), (3, 4, 512), (2, 4, 528),
]


@pytest.mark.parametrize("shape", STATIC_SHAPES)
def test_static_build_matches_oracle(pc, dev, shape):
    rng = np.random.default_rng(sum(shape))
    grid = scenegen.Grid(shape[2], shape[1], shape[0], 0.05)
    for p in (0.0, 0.003, 0.05, 0.5, 0.97, 1.0):
        occ = (rng.random(shape) < p).astype(np.uint8)
        say(f"static shape={shape} p={p}")
        ssq, sdf = gpu_static(pc, grid, occ, dev)
        rs, rf = oracle.build_static(grid, occ)
        np.testing.assert_array_equal(ssq.cpu().numpy(), rs)
        assert_f32_close(sdf.cpu().numpy(), rf)


@pytest.mark.parametrize("shape", [(6, 9, 64), (4, 5, 264)])
def test_static_build_unaligned_buffers(pc, dev, shape):
    """The x pass reads a row's occupancy as one 4-, 8- or 16-byte pack per
    lane and writes 16-byte packs when the buffers are aligned to them;
    an occupancy map starting at an odd byte and an output starting 4 bytes
    past a 16-byte boundary take the voxel-per-lane path: both give the
    oracle's bytes."""
    rng = np.random.default_rng(3)
    grid = scenegen.Grid(shape[2], shape[1], shape[0], 0.05)
    occ = (rng.random(shape) < 0.05).astype(np.uint8)
    rs, rf = oracle.build_static(grid, occ)
    V = occ.size
    flat = torch.zeros(V + 1, dtype=torch.uint8, device=dev)
    flat[1:] = to_dev(occ.reshape(-1), dev)
    occ_odd = flat[1:].view(shape)
    out = torch.empty(V + 1, dtype=torch.int32, device=dev)
    ssq_off = out[1:].view(shape)
    for o, q in ((occ_odd, None), (to_dev(occ, dev), ssq_off),
                 (occ_odd, ssq_off)):
        say(f"static unaligned shape={shape} occ+{o.data_ptr() % 16} "
            f"ssq+{(q.data_ptr() % 16) if q is not None else 0}")
        ssq, sdf = pc.build_static_sdf(grid, o, ssq=q)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(ssq.cpu().numpy(), rs)
        assert_f32_close(sdf.cpu().numpy(), rf)


@pytest.mark.parametrize("shape", [(4, 1024, 3), (700, 5, 40)])
def test_static_build_long_columns(pc, dev, shape):
    # Columns longer than one workgroup's LDS can hold take the path with
    # stacks in workspace memory.
    rng = np.random.default_rng(7)
    grid = scenegen.Grid(shape[2], shape[1], shape[0], 0.05)
    occ = (rng.random(shape) < 0.01).astype(np.uint8)
    say(f"static long columns shape={shape}")
    ssq, sdf = gpu_static(pc, grid, occ, dev)
    rs, rf = oracle.build_static(grid, occ)
    np.testing.assert_array_equal(ssq.cpu().numpy(), rs)


@pytest.mark.parametrize("shape", [(37, 29, 67), (600, 9, 40), (29, 131, 67)])
def test_static_build_every_segment_count(pc, dev, shape):
    """The column passes split each column into 1, 2, 4 or 8 segments (one
    wave each); every count gives the oracle's bytes, also when the column
    length is not a multiple of the count and when the segments' stacks
    need more than 64 KB of LDS (600-voxel columns)."""
    rng = np.random.default_rng(11)
    grid = scenegen.Grid(shape[2], shape[1], shape[0], 0.05)
    occ = (rng.random(shape) < 0.02).astype(np.uint8)
    rs, rf = oracle.build_static(grid, occ)
    occ_d = to_dev(occ, dev)
    h = pc.Handle()
    try:
        for S in (1, 2, 4, 8):
            say(f"static segments shape={shape} S={S}")
            h.set_tuning({"static_segments": S})
            ssq, sdf = pc.build_static_sdf(grid, occ_d, handle=h)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(ssq.cpu().numpy(), rs)
            assert_f32_close(sdf.cpu().numpy(), rf)
    finally:
        h.close()


def test_static_build_cube64_and_fp32_exact(pc, dev):
    sc = scenegen.cube64()
    ssq, sdf = gpu_static(pc, sc.grid, sc.occ, dev)
    rs, rf = oracle.build_static(sc.grid, sc.occ)
    np.testing.assert_array_equal(ssq.cpu().numpy(), rs)
    # correctly rounded sqrt on both sides: the fp32 field is bit-identical
    np.testing.assert_array_equal(sdf.cpu().numpy(), rf)


# --------------------------------------------------------------- composite

def run_composite(pc, sc, dev, want_ssq=True, want_sdf=True):
    ssq_s, _ = gpu_static(pc, sc.grid, sc.occ, dev)
    c, cf = pc.predicted_composite_sdf(sc.grid, ssq_s, sc.human_xy,
                                       sc.radius, sc.height,
                                       want_ssq=want_ssq, want_sdf=want_sdf)
    torch.cuda.synchronize()
    return ssq_s, c, cf


def check_composite(pc, sc, dev):
    say(f"composite {sc.name} grid={sc.grid.nx}x{sc.grid.ny}x{sc.grid.nz} "
        f"n={sc.n_slices} K={sc.n_humans} r={sc.radius} H={sc.height}")
    _, c, cf = run_composite(pc, sc, dev)
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                        sc.height)
    np.testing.assert_array_equal(c.cpu().numpy(), wc)
    assert_f32_close(cf.cpu().numpy(), wf)


@pytest.mark.parametrize("seed,dims,K,n", [
    (1, (33, 27, 21), 3, 4), (2, (67, 131, 29), 2, 3), (3, (64, 64, 40), 8, 2),
    (4, (5, 7, 3), 1, 2), (5, (130, 70, 33), 4, 5), (6, (1, 40, 40), 2, 2),
    (7, (40, 1, 40), 2, 2), (8, (257, 65, 9), 3, 2),
    # 16 x (2 x 7 + 1) = 240 words of centres and radii, the most the
    # planar kernels take in their arguments; 17 slices are uploaded
    (9, (30, 41, 12), 7, 16), (10, (30, 41, 12), 7, 17)])
def test_composite_small_scenes(pc, dev, seed, dims, K, n):
    sc = scenegen.small_scene(seed, *dims, h=0.05, n_boxes=5, n_humans=K,
                              n_slices=n)
    check_composite(pc, sc, dev)


@pytest.mark.parametrize("seed,dims,K,n", [
    (11, (1024, 1024, 3), 5, 2),   # the largest plane the interface takes
    (12, (1024, 9, 5), 3, 2), (13, (7, 1024, 6), 4, 2)])
def test_composite_maximum_axis_lengths(pc, dev, seed, dims, K, n):
    """Axes of 1024 voxels (the interface's limit): chord tables and row
    passes of 1024 rows or columns, planes of a million pixels."""
    sc = scenegen.small_scene(seed, *dims, h=0.02, n_boxes=5, n_humans=K,
                              n_slices=n)
    say(f"composite maximum axes dims={dims} K={K} n={n}")
    check_composite(pc, sc, dev)


def width_case_scene(dims):
    """Scenes for the composite's pack shapes.  Planes of fewer than four
    pixels get one free-standing human on a nearly empty grid, tall enough
    to end inside it, so that every layer (and every layer boundary a pack
    crosses) has its own value."""
    nx, ny, nz = dims
    if nx * ny >= 4:
        return scenegen.small_scene(21, nx, ny, nz, h=0.05, n_boxes=5,
                                    n_humans=3, n_slices=3)
    sc = scenegen.small_scene(22, nx, ny, nz, h=0.25, n_boxes=1, n_humans=1,
                              n_slices=3, height=0.6)
    ext = sc.grid.extent
    sc.occ[:] = 0
    sc.occ[-1, 0, 0] = 1
    sc.human_xy = np.array([[[(0.3 + 0.3 * s) * ext[0], 0.5 * ext[1]]]
                            for s in range(3)])
    return sc


@pytest.mark.parametrize("dims", [
    (21, 60, 17), (130, 70, 9),   # 4-wide, nx odd / nx = 2 mod 4
    (34, 27, 13),                 # 2-wide planar packs (V = 2 mod 4)
    (33, 27, 20), (34, 27, 12),   # 4-wide streams, planar values gathered
    (33, 27, 22),                 # 2-wide streams, gathered
    (33, 27, 21),                 # 1-wide (V odd)
    (1, 1, 8), (3, 1, 4), (2, 1, 6),  # planes smaller than a pack
    (3, 1, 1), (1, 1, 7), (3, 1, 2)])  # V of 3, 7 and 6 voxels
@pytest.mark.parametrize("offset", [0, 1, 2])
@pytest.mark.parametrize("copy", [1, 2])
def test_composite_vector_widths_and_alignment(pc, dev, dims, offset, copy):
    """The composite streams 4, 2 or 1 voxels per lane by V mod 4 and the
    alignment of its three buffers, reading the planar values as one
    vector when the pack width divides nx*ny and one by one otherwise
    (a pack may then cross layer boundaries).  Buffers offset by one or two
    elements (4- and 8-byte aligned) take the narrower packs.  Each pack
    width reads the static values from the int32 field (copy 1) or from
    the 16-bit copy (copy 2).  Every case gives the oracle's bytes."""
    sc = width_case_scene(dims)
    say(f"composite widths grid={dims} offset={offset} static16={copy}")
    n, V = sc.n_slices, sc.grid.nvox
    shp = (n,) + sc.grid.shape_zyx
    ssq_s, _ = gpu_static(pc, sc.grid, sc.occ, dev)
    bs = torch.empty(V + offset, dtype=torch.int32, device=dev)
    bs[offset:] = ssq_s.reshape(-1)
    bi = torch.empty(n * V + offset, dtype=torch.int32, device=dev)
    bf = torch.empty(n * V + offset, dtype=torch.float32, device=dev)
    oc, of = bi[offset:].view(shp), bf[offset:].view(shp)
    h = pc.Handle()
    try:
        h.set_tuning({"composite_static16": copy})
        pc.predicted_composite_sdf(sc.grid,
                                   bs[offset:].view(sc.grid.shape_zyx),
                                   sc.human_xy, sc.radius, sc.height,
                                   out_ssq=oc, out_sdf=of, handle=h)
        torch.cuda.synchronize()
    finally:
        h.close()
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                        sc.height)
    assert np.unique(wc).size > 2  # the case has structure to get wrong
    np.testing.assert_array_equal(oc.cpu().numpy(), wc)
    assert_f32_close(of.cpu().numpy(), wf)


def far_scene(kind):
    """Static fields beyond the 16-bit copy's range (|value| > 32767):
    free voxels up to 399 voxels from the nearest obstacle, an empty map
    (+inf everywhere) and a full one (-inf everywhere), 8 slices."""
    sc = scenegen.small_scene(31, 400, 12, 10, h=0.05, n_boxes=1,
                              n_humans=2, n_slices=8)
    sc.occ[:] = 0
    if kind == "far":
        sc.occ[2:5, 3:6, 0:3] = 1   # obstacle at x = 0..2, z = 2..4
    elif kind == "full":
        sc.occ[:] = 1
    return sc


@pytest.mark.parametrize("kind", ["far", "empty", "full"])
def test_composite_static16_far_values(pc, dev, kind):
    """The 16-bit static copy holds values in [-32767, 32767] and sends
    the composite to the int32 field for every other one: with the copy
    forced, left to the library (not used on a grid this small) and off,
    the oracle's bytes on fields whose values mostly lie beyond that
    range."""
    sc = far_scene(kind)
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    if kind == "far":
        assert (rs > 32767).sum() > sc.grid.nvox // 4
    wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                        sc.height)
    ssq_s, _ = gpu_static(pc, sc.grid, sc.occ, dev)
    for copy in (2, 0, 1):
        say(f"composite static16={copy} {kind}")
        h = pc.Handle()
        try:
            h.set_tuning({"composite_static16": copy})
            c, cf = pc.predicted_composite_sdf(sc.grid, ssq_s, sc.human_xy,
                                               sc.radius, sc.height, handle=h)
            torch.cuda.synchronize()
        finally:
            h.close()
        np.testing.assert_array_equal(c.cpu().numpy(), wc)
        assert_f32_close(cf.cpu().numpy(), wf)


@pytest.mark.parametrize("r,H", [(0.25, 1.8), (0.0, 1.8), (0.25, 0.01),
                                 (0.25, 0.0249), (0.25, 0.025), (0.6, 100.0),
                                 (5.0, 0.5), (5.0, 100.0), (0.07, 0.3)])
def test_composite_cylinder_edge_cases(pc, dev, r, H):
    # radius 0, no layer under the top, one layer, the whole column, a disk
    # covering the whole plane (no free voxel in the plane), both at once.
    sc = scenegen.small_scene(11, 37, 29, 23, h=0.05, n_boxes=4, n_humans=3,
                              n_slices=3, radius=r, height=H)
    check_composite(pc, sc, dev)


def test_composite_no_humans_and_empty_static(pc, dev):
    sc = scenegen.small_scene(12, 20, 18, 16, n_boxes=3, n_humans=2,
                              n_slices=2)
    sc.human_xy = np.zeros((2, 0, 2))
    check_composite(pc, sc, dev)
    sc2 = scenegen.small_scene(13, 20, 18, 16, n_boxes=3, n_humans=2,
                               n_slices=2)
    sc2.occ[:] = 0
    check_composite(pc, sc2, dev)
    sc2.human_xy[:] = -100.0  # everyone outside: the whole field is +inf
    check_composite(pc, sc2, dev)
    sc3 = scenegen.small_scene(14, 20, 18, 16, n_boxes=3, n_humans=1,
                               n_slices=1)
    sc3.occ[:] = 1            # full static grid: -inf everywhere
    check_composite(pc, sc3, dev)


@pytest.mark.parametrize("dims", [(36, 30, 20), (35, 29, 21)])
def test_composite_single_output_modes(pc, dev, dims):
    # 35 x 29 x 21 has odd V (the flattened-pack kernels, one per output
    # mode) and 3 V = 1 mod 4 (a partial last pack)
    say(f"composite single outputs {dims}")
    sc = scenegen.small_scene(15, *dims, n_humans=2, n_slices=3)
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                        sc.height)
    _, c, cf = run_composite(pc, sc, dev, want_sdf=False)
    assert cf is None
    np.testing.assert_array_equal(c.cpu().numpy(), wc)
    _, c, cf = run_composite(pc, sc, dev, want_ssq=False)
    assert c is None
    assert_f32_close(cf.cpu().numpy(), wf)


def test_composite_cube64(pc, dev):
    check_composite(pc, scenegen.cube64(), dev)


@pytest.fixture(scope="module")
def room256_ref():
    sc = scenegen.room256()
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                        sc.height)
    return sc, wc, wf


@pytest.mark.slow
def test_composite_room256_full(pc, dev, room256_ref):
    """The full 256x256x128 x 20-slice workload, element by element."""
    sc, wc, wf = room256_ref
    say("composite room256 full")
    _, c, cf = run_composite(pc, sc, dev)
    np.testing.assert_array_equal(c.cpu().numpy(), wc)
    assert_f32_close(cf.cpu().numpy(), wf)


@pytest.mark.slow
@pytest.mark.parametrize("G,order,copy", [
    (1, 0, 0), (3, 0, 0), (5, 0, 0), (10, 0, 0), (20, 0, 0), (1, 1, 0),
    (2, 1, 0), (3, 1, 0), (20, 1, 0), (2, 0, 1), (1, 0, 2), (2, 0, 2),
    (1, 1, 2), (10, 0, 2), (20, 1, 2)])
def test_composite_room256_every_slice_group(pc, dev, room256_ref, G, order,
                                             copy):
    """The same workload in the other launch shapes the autotuner chooses
    between (slices per block row, block order) and with the 16-bit static
    copy left to the library (not used on this grid), off or forced: the
    oracle's bytes in each."""
    sc, wc, wf = room256_ref
    say(f"composite room256 with {G} slices per block row, order {order}, "
        f"static16 {copy}")
    occ_d = to_dev(sc.occ.astype(np.uint8), dev)
    h = pc.Handle()
    try:
        h.set_tuning({"composite_slices_per_block": G,
                      "composite_order": order,
                      "composite_static16": copy})
        ssq_s, _ = pc.build_static_sdf(sc.grid, occ_d, want_sdf=False,
                                       handle=h)
        c, cf = pc.predicted_composite_sdf(sc.grid, ssq_s, sc.human_xy,
                                           sc.radius, sc.height, handle=h)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(c.cpu().numpy(), wc)
        assert_f32_close(cf.cpu().numpy(), wf)
    finally:
        h.close()


def test_composite_deterministic_and_on_side_stream(pc, dev):
    sc = scenegen.small_scene(16, 96, 64, 48, n_humans=3, n_slices=4)
    _, c1, f1 = run_composite(pc, sc, dev)
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        _, c2, f2 = run_composite(pc, sc, dev)
    s.synchronize()
    assert torch.equal(c1, c2) and torch.equal(f1, f2)


# ------------------------------------------------------------------ queries

def check_queries(pc, sc, dev, centre, radius, slices, eps=0.3):
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    _, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                       sc.height)
    wd, wg, wst, wc = oracle.query(sc.grid, wf, centre, radius, slices,
                                   hinge_eps=eps)
    _, _, cf = run_composite(pc, sc, dev, want_ssq=False)
    d, g, st, cost = pc.query_spheres(sc.grid, cf, to_dev(centre, dev),
                                      to_dev(radius, dev),
                                      to_dev(slices, dev), hinge_eps=eps,
                                      want_cost=True)
    torch.cuda.synchronize()
    d, g, st, cost = (x.cpu().numpy() for x in (d, g, st, cost))
    np.testing.assert_array_equal(st, wst)
    h = sc.grid.h
    for got, want, floor in ((d, wd, h), (cost, wc, h)):
        nanw = np.isnan(want)
        assert (np.isnan(got) == nanw).all()
        fin = np.isfinite(want)
        np.testing.assert_array_equal(got[~fin & ~nanw], want[~fin & ~nanw])
        err = np.abs(got[fin].astype(np.float64) - want[fin])
        assert (err <= 1e-6 * np.maximum(np.abs(want[fin]), floor)).all()
    nanw = np.isnan(wg)
    assert (np.isnan(g) == nanw).all()
    err = np.abs(g[~nanw].astype(np.float64) - wg[~nanw])
    assert (err <= 1e-6 * np.maximum(np.abs(wg[~nanw]), 1.0)).all()


def test_queries_room256(pc, dev):
    sc = scenegen.room256()
    q = sc.queries
    say("queries room256 Q=", len(q.radius))
    check_queries(pc, sc, dev, q.centre, q.radius, q.slice)


def test_queries_edge_cases(pc, dev):
    sc = scenegen.small_scene(21, 40, 36, 30, h=0.05, n_humans=2, n_slices=3)
    rng = np.random.default_rng(5)
    Q = 3000
    L = np.array(sc.grid.extent)
    centre = (rng.uniform(-0.2, 1.2, size=(Q, 3)) * L).astype(np.float32)
    # exact voxel centres and the last cell face
    centre[:50] = ((rng.integers(0, 30, size=(50, 3)) + 0.5) *
                   sc.grid.h).astype(np.float32)
    centre[50] = (L - sc.grid.h / 2).astype(np.float32)
    radius = rng.uniform(0.05, 0.15, Q).astype(np.float32)
    slices = rng.integers(-2, 6, Q).astype(np.int32)
    check_queries(pc, sc, dev, centre, radius, slices)


def test_queries_infinite_fields(pc, dev):
    sc = scenegen.small_scene(22, 10, 9, 8, n_humans=1, n_slices=1)
    sc.occ[:] = 0
    sc.human_xy[:] = -50.0
    c = np.array([[0.2, 0.2, 0.2], [0.1, 0.3, 0.2]], np.float32)
    check_queries(pc, sc, dev, c, np.zeros(2, np.float32),
                  np.zeros(2, np.int32))
    sc.occ[:] = 1
    check_queries(pc, sc, dev, c, np.zeros(2, np.float32),
                  np.zeros(2, np.int32))

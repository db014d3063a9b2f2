"""The rows after the hot path proper: the full recompute per slice (the
baseline of the paper's composite benchmark) and cylinders whose radius
grows with the prediction time (the discussion section's proposal), both
against the oracle."""
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
    return m


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


CASES = [(71, (37, 29, 23), 3, 2), (72, (64, 48, 40), 4, 3),
         (73, (21, 60, 17), 1, 1), (74, (8, 8, 8), 2, 0)]


@pytest.mark.parametrize("seed,dims,n,K", CASES)
def test_recompute_matches_oracle(pc, dev, seed, dims, n, K):
    sc = scenegen.small_scene(seed, *dims, h=0.05, n_humans=K, n_slices=n)
    say(f"recompute seed={seed} dims={dims} n={n} K={K}")
    occ = to_dev(sc.occ, dev)
    ssq, sdf = pc.recompute_sdf(sc.grid, occ, sc.human_xy, sc.radius,
                                sc.height)
    s_ssq, _ = pc.build_static_sdf(sc.grid, occ)
    c, _ = pc.predicted_composite_sdf(sc.grid, s_ssq, sc.human_xy, sc.radius,
                                      sc.height)
    torch.cuda.synchronize()
    ssq, sdf, c = ssq.cpu().numpy(), sdf.cpu().numpy(), c.cpu().numpy()
    for j in range(n):
        hum = oracle.human_occupancy(sc.grid, sc.human_xy[j], sc.radius,
                                     sc.height)
        union = np.maximum(sc.occ, hum)
        want = oracle.signed_sq(union)
        np.testing.assert_array_equal(ssq[j], want)
        np.testing.assert_array_equal(sdf[j], oracle.to_float(want,
                                                              sc.grid.h))
        # outside every obstacle the composite is the union's field
        free = union == 0
        np.testing.assert_array_equal(c[j][free], ssq[j][free])
        assert ((c[j] < 0) == (union != 0)).all()


@pytest.mark.parametrize("seed,dims,n,K", CASES[:3])
def test_growing_radius_matches_oracle(pc, dev, seed, dims, n, K):
    sc = scenegen.small_scene(seed, *dims, h=0.05, n_humans=K, n_slices=n)
    # r(t) = r0 + sigma t with t = j dt; the first slice also at radius 0
    rad = 0.25 + 0.3 * np.arange(n) * sc.dt
    rad[0] = 0.0 if n > 1 else rad[0]
    say(f"growing radius seed={seed} dims={dims} radii={rad}")
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    s_ssq, _ = pc.build_static_sdf(sc.grid, to_dev(sc.occ, dev))
    c, cf = pc.predicted_composite_sdf_growing(sc.grid, s_ssq, sc.human_xy,
                                               rad, sc.height)
    torch.cuda.synchronize()
    c, cf = c.cpu().numpy(), cf.cpu().numpy()
    for j in range(n):
        wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy[j:j + 1],
                                            rad[j], sc.height)
        np.testing.assert_array_equal(c[j], wc[0])
        np.testing.assert_array_equal(cf[j], wf[0])


@pytest.mark.parametrize("seed,dims,n,K", CASES)
def test_template_matches_oracle(pc, dev, seed, dims, n, K):
    from oracle.template import template_composite
    sc = scenegen.small_scene(seed, *dims, h=0.05, n_humans=K, n_slices=n)
    say(f"template seed={seed} dims={dims} n={n} K={K}")
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    s_ssq, _ = pc.build_static_sdf(sc.grid, to_dev(sc.occ, dev))
    c, cf = pc.template_composite_sdf(sc.grid, s_ssq, sc.human_xy,
                                      sc.radius, sc.height)
    torch.cuda.synchronize()
    wc, wf = template_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                sc.height)
    np.testing.assert_array_equal(c.cpu().numpy(), wc)
    np.testing.assert_array_equal(cf.cpu().numpy(), wf)


def test_template_whole_voxel_motion_equals_exact(pc, dev):
    sc = scenegen.small_scene(75, 48, 40, 30, h=0.05, n_boxes=5,
                              n_humans=2, n_slices=6)
    h = sc.grid.h
    start = np.array([[10.3 * h, 12.6 * h], [33.1 * h, 24.4 * h]])
    step = np.array([[2, 1], [-1, -2]]) * h
    xy = start[None] + np.arange(6)[:, None, None] * step[None]
    say("template whole-voxel motion")
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    s_ssq, _ = pc.build_static_sdf(sc.grid, to_dev(sc.occ, dev))
    c, cf = pc.template_composite_sdf(sc.grid, s_ssq, xy, 0.2, 0.9)
    e, ef = pc.predicted_composite_sdf(sc.grid, s_ssq, xy, 0.2, 0.9)
    torch.cuda.synchronize()
    wc, wf = oracle.predicted_composite(sc.grid, rs, xy, 0.2, 0.9)
    np.testing.assert_array_equal(c.cpu().numpy(), wc)
    np.testing.assert_array_equal(cf.cpu().numpy(), wf)
    np.testing.assert_array_equal(e.cpu().numpy(), wc)


@pytest.mark.parametrize("seed,S,J", [(91, 20, 30), (92, 7, 1), (93, 45, 130)])
def test_obstacle_factors_match_oracle(pc, dev, seed, S, J):
    from oracle.factors import obstacle_factors
    sc = scenegen.small_scene(seed, 40, 36, 30, h=0.05, n_humans=2,
                              n_slices=5)
    rng = np.random.default_rng(seed)
    L = np.array(sc.grid.extent)
    c = (rng.uniform(-0.05, 1.05, size=(S, J, 3)) * L).astype(np.float32)
    r = rng.uniform(0.02, 0.15, size=J).astype(np.float32)
    sl = rng.integers(-1, sc.n_slices + 3, size=S).astype(np.int32)
    eps, sigma = 0.3, 0.08
    say(f"obstacle factors seed={seed} S={S} J={J}")
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    _, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                       sc.height)
    werr, wjac, wcost = obstacle_factors(sc.grid, wf, c, r, sl, eps, sigma)
    s_ssq, _ = pc.build_static_sdf(sc.grid, to_dev(sc.occ, dev))
    _, cf = pc.predicted_composite_sdf(sc.grid, s_ssq, sc.human_xy,
                                       sc.radius, sc.height, want_ssq=False)
    err, jac, cost = pc.obstacle_factors(sc.grid, cf, to_dev(c, dev),
                                         to_dev(r, dev), to_dev(sl, dev), eps,
                                         sigma)
    torch.cuda.synchronize()
    err, jac, cost = err.cpu().numpy(), jac.cpu().numpy(), cost.cpu().numpy()
    nan = np.isnan(werr)
    assert (np.isnan(err) == nan).all()
    fin = ~nan & np.isfinite(werr)
    e = np.abs(err[fin].astype(np.float64) - werr[fin])
    assert (e <= 1e-6 * np.maximum(np.abs(werr[fin]), sc.grid.h)).all()
    jn = np.isnan(wjac)
    assert (np.isnan(jac) == jn).all()
    e = np.abs(jac[~jn].astype(np.float64) - wjac[~jn])
    assert (e <= 1e-6 * np.maximum(np.abs(wjac[~jn]), 1.0)).all()
    cn = ~np.isfinite(wcost)
    assert (np.isnan(cost) == np.isnan(wcost)).all()
    np.testing.assert_allclose(cost[~cn], wcost[~cn], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("seed,dims,zr", [(95, (37, 29, 23), (0, 22)),
                                          (96, (64, 48, 40), (3, 17)),
                                          (97, (5, 70, 9), (8, 8))])
def test_floor_sdf_matches_oracle(pc, dev, seed, dims, zr):
    sc = scenegen.small_scene(seed, *dims, h=0.05, n_boxes=8)
    say(f"floor sdf seed={seed} dims={dims} layers={zr}")
    ssq, sdf = pc.build_floor_sdf(sc.grid, to_dev(sc.occ, dev), *zr)
    torch.cuda.synchronize()
    flat = sc.occ[zr[0]:zr[1] + 1].any(0).astype(np.uint8)
    want = oracle.signed_sq(flat[None])[0]
    np.testing.assert_array_equal(ssq.cpu().numpy(), want)
    np.testing.assert_array_equal(sdf.cpu().numpy(),
                                  oracle.to_float(want, sc.grid.h))


def _queries(sc, Q, seed):
    rng = np.random.default_rng(seed)
    L = np.array(sc.grid.extent)
    c = (rng.uniform(-0.1, 1.1, size=(Q, 3)) * L).astype(np.float32)
    r = rng.uniform(0.0, 0.15, size=Q).astype(np.float32)
    s = rng.integers(-1, sc.n_slices + 2, size=Q).astype(np.int32)
    return c, r, s


@pytest.mark.parametrize("seed,dims,n,K", CASES)
def test_direct_queries_match_oracle_and_fields(pc, dev, seed, dims, n, K):
    sc = scenegen.small_scene(seed, *dims, h=0.05, n_humans=K, n_slices=n)
    c, r, s = _queries(sc, 3000, seed)
    say(f"direct queries seed={seed} dims={dims} n={n} K={K}")
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    _, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                       sc.height)
    wd, wg, wst, wc = oracle.query(sc.grid, wf, c, r, s, hinge_eps=0.3)
    s_ssq, _ = pc.build_static_sdf(sc.grid, to_dev(sc.occ, dev))
    cd, rd, sd = to_dev(c, dev), to_dev(r, dev), to_dev(s, dev)
    d, g, st, cost = pc.query_spheres_direct(
        sc.grid, s_ssq, sc.human_xy, sc.radius, sc.height, cd, rd, sd,
        hinge_eps=0.3, want_cost=True)
    _, cf = pc.predicted_composite_sdf(sc.grid, s_ssq, sc.human_xy,
                                       sc.radius, sc.height, want_ssq=False)
    fd, fg, fst, fc = pc.query_spheres(sc.grid, cf, cd, rd, sd, hinge_eps=0.3,
                                       want_cost=True)
    torch.cuda.synchronize()
    d, g, st, cost = (t.cpu().numpy() for t in (d, g, st, cost))
    # bit-identical to sampling the built fields
    for a, b in zip((d, g, st, cost), (fd, fg, fst, fc)):
        np.testing.assert_array_equal(a, b.cpu().numpy())
    # and to the oracle within the query contract
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
    err = np.abs(g[~nanw].astype(np.float64) - wg[~nanw])
    assert (err <= 1e-6 * np.maximum(np.abs(wg[~nanw]), 1.0)).all()


def test_direct_queries_room256_bit_identical(pc, dev):
    sc = scenegen.room256()
    q = sc.queries
    say("direct queries room256, 10k")
    s_ssq, _ = pc.build_static_sdf(sc.grid, to_dev(sc.occ, dev))
    cd, rd, sd = to_dev(q.centre, dev), to_dev(q.radius, dev), \
        to_dev(q.slice, dev)
    d, g, st, _ = pc.query_spheres_direct(sc.grid, s_ssq, sc.human_xy,
                                          sc.radius, sc.height, cd, rd, sd)
    _, cf = pc.predicted_composite_sdf(sc.grid, s_ssq, sc.human_xy,
                                       sc.radius, sc.height, want_ssq=False)
    fd, fg, fst, _ = pc.query_spheres(sc.grid, cf, cd, rd, sd)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(d.cpu().numpy(), fd.cpu().numpy())
    np.testing.assert_array_equal(g.cpu().numpy(), fg.cpu().numpy())
    np.testing.assert_array_equal(st.cpu().numpy(), fst.cpu().numpy())

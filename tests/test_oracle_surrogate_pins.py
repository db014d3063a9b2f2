"""Pins of the per-human surrogate's oracle by cases whose answer is known
without it: the features against geometry computed another way (nearest
point of the solid cylinder, lattice identities), the gradient chain
against central differences, the residual's range against the exact
single-human field, and the combination rule against the exact query when
the network reproduces every human's exact field (the band rule makes the
two agree to rounding), a constant network (closed form), an infinite
margin (the exact query), a non-finite network, absent and clipped humans.
CPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from oracle import surrogate as osur


def room(seed=41, nx=30, ny=26, nz=14, h=0.05, K=3, n=3, boxes=4):
    sc = scenegen.small_scene(seed, nx, ny, nz, h=h, n_boxes=boxes,
                              n_humans=K, n_slices=n, radius=0.2,
                              height=0.45)
    rs, rf = oracle.build_static(sc.grid, sc.occ)
    _, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                       sc.height)
    return sc, rf, wf


def queries(sc, Q=600, seed=0, lo=-0.05, hi=1.05):
    rng = np.random.default_rng(seed)
    L = np.array(sc.grid.extent)
    c = (rng.uniform(lo, hi, size=(Q, 3)) * L).astype(np.float32)
    r = rng.uniform(0, 0.1, size=Q).astype(np.float32)
    s = rng.integers(-1, sc.n_slices + 2, size=Q).astype(np.int32)
    return c, r, s


def geometry(sc, c, s, k):
    g, _ = osur.lattice(sc.grid, c)
    G = osur.human_geometry(sc.grid, sc.human_xy, sc.radius, sc.height, g,
                            s, np.full(len(s), k))
    return g, G


def test_features_against_cylinder_geometry():
    sc, _, _ = room()
    c, _, s = queries(sc, Q=2000, lo=0.0, hi=1.0)
    h = sc.grid.h
    Kt = osur.top_layer(sc.grid, sc.height)
    # the top layer is the last whose centre lies at or under the top
    assert (Kt + 0.5) * h <= sc.height < (Kt + 1.5) * h
    for k in range(sc.n_humans):
        g, G = geometry(sc, c, s, k)
        x = osur.features(G, g, np.float64)
        # the axis in voxel coordinates, from the metres directly
        p = sc.human_xy[np.clip(s, 0, sc.n_slices - 1), k]
        ax = (p - np.array(sc.grid.origin[:2])) / h - 0.5
        np.testing.assert_allclose(g[:, 0] - x[:, 0] * G["rho"], ax[:, 0],
                                   atol=2e-5)
        # d: distance from g to the nearest point of the solid cylinder
        # {|xy - axis| <= Rv, z <= Kt}
        Rv = sc.radius / h
        v = g[:, :2] - ax
        rho = np.linalg.norm(v, axis=1)
        near = ax + v * (np.minimum(rho, Rv) / np.maximum(rho, 1e-300))[:,
                                                                       None]
        nz = np.minimum(g[:, 2], Kt)
        d = np.sqrt(np.sum((g[:, :2] - near) ** 2, axis=1) +
                    (g[:, 2] - nz) ** 2)
        np.testing.assert_allclose(x[:, 4], d, atol=2e-4)
        # unit direction, and 1/(1+d)
        np.testing.assert_allclose(x[:, 0] ** 2 + x[:, 1] ** 2, 1.0,
                                   atol=1e-12)
        np.testing.assert_allclose(x[:, 5] * (1 + x[:, 4]), 1.0, atol=1e-12)
        # phases: the axis minus its phase lies on the lattice, as does
        # the query minus its phase
        X = osur._fixed(p[:, 0], sc.grid.origin[0], h)
        cx = X / 65536.0 - 0.5
        phx = np.arctan2(x[:, 6], x[:, 7]) / (2 * np.pi) % 1.0
        fr = cx - phx
        assert np.all(np.abs(fr - np.round(fr)) < 1e-9)
        fgz = np.arctan2(x[:, 14], x[:, 15]) / (2 * np.pi) % 1.0
        fr = g[:, 2] - fgz
        assert np.all(np.abs(fr - np.round(fr)) < 1e-9)


def test_gradient_chain_against_central_differences():
    """With a network linear in the features (value w.x, input gradient
    w), the gradient equals the central differences of the prediction in
    metres, y(c) = h (d + w.x) with g = (c - o)/h - 1/2, taken in metres,
    at points away from the kinks (the disk's rim, the top, cell
    faces)."""
    sc, _, _ = room(K=1)
    rng = np.random.default_rng(5)
    w = rng.normal(size=16) * 0.05
    c, _, s = queries(sc, Q=3000, lo=0.0, hi=1.0, seed=3)
    h = sc.grid.h
    g, G = geometry(sc, c, s, 0)
    f = g - np.floor(g)
    ok = (np.abs(G["a"]) > 0.05) & (np.abs(G["w"]) > 0.05) & \
        np.all((f > 0.01) & (f < 0.99), axis=1) & (G["rho"] > 0.5)
    ok &= s >= 0
    assert ok.sum() > 500
    x = osur.features(G, g, np.float64)
    delta = np.clip(x @ w, osur.RES_LO, osur.RES_HI)
    keep = ok & (np.abs(x @ w) < 0.4)
    _, grad = osur.value_and_gradient(G, g, h, (x @ w).astype(np.float32),
                                      np.tile(w.astype(np.float32),
                                              (len(s), 1)))
    eps = 1e-5 * h  # metres
    o = np.asarray(sc.grid.origin, np.float64)
    cm = (g + 0.5) * h + o  # the centres in metres (fp64)

    def y_m(cc):
        gg = (cc - o) / h - 0.5
        GG = osur.human_geometry(sc.grid, sc.human_xy, sc.radius, sc.height,
                                 gg, s, np.zeros(len(s), np.int64))
        return h * (GG["d"] + osur.features(GG, gg, np.float64) @ w)
    for a in range(3):
        e = np.zeros(3)
        e[a] = eps
        fd = (y_m(cm + e) - y_m(cm - e)) / (2 * eps)
        np.testing.assert_allclose(grad[keep, a], fd[keep], rtol=1e-4,
                                   atol=1e-4)
    assert np.all(np.isfinite(delta))


def test_residual_range_of_the_exact_single_human_field():
    """The exact field of one human (the composite over an empty room) is
    at least the distance d to the continuous cylinder (every occupied
    voxel centre lies in the cylinder, and the trilinear sample of a
    convex function's samples is at least the function) and exceeds it by
    about one voxel at most (the voxelised disk's rim lies up to a voxel
    inside the circle): the clamp [-1/2, 3/2] of the residual holds every
    exact value with room to spare."""
    for seed, h, r in ((7, 0.05, 0.2), (8, 0.02, 0.25), (9, 0.04, 0.31)):
        sc = scenegen.small_scene(seed, 40, 36, 20, h=h, n_boxes=0,
                                  n_humans=1, n_slices=3, radius=r,
                                  height=12 * h)
        # whole disks at three random sub-voxel phases
        rng = np.random.default_rng(seed)
        L = np.array(sc.grid.extent[:2])
        sc.human_xy = rng.uniform(r + 2 * h, L - r - 2 * h, size=(3, 1, 2))
        empty = np.full(sc.grid.shape_zyx, np.iinfo(np.int32).max, np.int32)
        _, wf = oracle.predicted_composite(sc.grid, empty, sc.human_xy,
                                           sc.radius, sc.height)
        c, _, s = queries(sc, Q=4000, lo=0.0, hi=1.0, seed=seed)
        s = np.abs(s) % sc.n_slices
        ex, _, _, _ = oracle.query(sc.grid, wf, c, np.zeros(len(s)), s)
        g, G = geometry(sc, c, s, 0)
        _, inside = osur.lattice(sc.grid, c)
        # whole disks (clipped ones are farther) and centres within the
        # span of voxel centres (the exact query clamps the others)
        far = G["present"] & ~G["clipped"] & inside & (G["d"] >= 1.0) & \
            np.isfinite(ex)
        res = ex[far] / h - G["d"][far]
        assert far.sum() > 500
        assert res.min() >= -1e-5 and res.max() < 1.25, (res.min(),
                                                         res.max())


def exact_network(sc, c, s):
    """A 'network' returning, for human k's rows, the residual of that
    human's exact single-human field at each query (its composite over an
    empty room), with zero input gradient."""
    g, _ = osur.lattice(sc.grid, c)
    empty = np.full(sc.grid.shape_zyx, np.iinfo(np.int32).max, np.int32)
    cache = {}
    for k in range(sc.n_humans):
        _, wf = oracle.predicted_composite(sc.grid, empty,
                                           sc.human_xy[:, k:k + 1],
                                           sc.radius, sc.height)
        ex, _, _, _ = oracle.query(sc.grid, wf, c, np.zeros(len(s)),
                                   np.clip(s, 0, sc.n_slices - 1))
        _, G = geometry(sc, c, np.clip(s, 0, sc.n_slices - 1), k)
        with np.errstate(invalid="ignore"):
            cache[k] = (ex.astype(np.float64) / sc.grid.h - G["d"])

    def net(x, k):
        return cache[k].astype(np.float32), np.zeros((len(s), 16),
                                                     np.float32)
    return net


@pytest.mark.parametrize("seed", [41, 42, 43])
def test_exact_network_reproduces_the_exact_query(seed):
    """Every answered query equals the exact query (to fp32 rounding of
    the per-human values), so the min over candidates with the band rule
    is the trilinear sample of the composite; some are answered (the room is
    small: most of it lies within the band of a boundary),
    and dropping the band makes some answers differ."""
    sc, rf, wf = room(seed=seed)
    c, r, s = queries(sc, Q=3000, seed=seed, lo=0.0, hi=1.0)
    net = exact_network(sc, c, s)
    band = 2 * np.sqrt(3) * sc.grid.h
    d, g, st, cost, used = osur.query(sc.grid, wf, rf, net, sc.human_xy,
                                      sc.radius, sc.height, c, r, s,
                                      margin=0.02, band=band, hinge_eps=0.3)
    ed, eg, est, ecost = oracle.query(sc.grid, wf, c, r, s, hinge_eps=0.3)
    acc = (used == 0) & (s >= 0)
    assert acc.mean() > 0.15
    tol = 1e-6 * np.maximum(np.abs(ed[acc]), sc.grid.h) + 2e-7
    assert np.all(np.abs(d[acc] - ed[acc]) <= tol)
    np.testing.assert_array_equal(st[acc], est[acc])
    # without the band the min of the samples differs somewhere
    d0, _, _, _, u0 = osur.query(sc.grid, wf, rf, net, sc.human_xy,
                                 sc.radius, sc.height, c, r, s, margin=0.02,
                                 band=0.0)
    a0 = (u0 == 0) & (s >= 0)
    assert np.any(np.abs(d0[a0] - ed[a0]) > 1e-4)


def test_constant_network_closed_form():
    sc, rf, wf = room(seed=44, boxes=0)
    c, r, s = queries(sc, seed=1)
    dv = float(np.float32(0.37))  # the network's fp32 output

    def net(x, k):
        return (np.full(len(x), dv, np.float32),
                np.zeros((len(x), 16), np.float32))
    d, g, st, cost, used = osur.query(sc.grid, wf, rf, net, sc.human_xy,
                                      sc.radius, sc.height, c, r, s,
                                      margin=0.05, band=0.0, hinge_eps=0.3)
    h = sc.grid.h
    gq, inside = osur.lattice(sc.grid, c)
    best = np.full(len(s), np.inf, np.float32)
    for k in range(sc.n_humans):
        _, G = geometry(sc, c, s, k)
        yk = (h * (G["d"] + dv)).astype(np.float32)
        best = np.where(G["present"], np.minimum(best, yk), best)
    acc = (used == 0) & (s >= 0)
    assert acc.any()
    np.testing.assert_array_equal(d[acc], (best - r)[acc])
    assert np.all(inside[acc])
    neg = s < 0
    assert np.isnan(d[neg]).all() and (st[neg] == 32).all()
    assert (used[neg] == 0).all()


def test_infinite_margin_is_the_exact_query():
    sc, rf, wf = room(seed=45)
    c, r, s = queries(sc, seed=2)
    net = osur.network(np.random.default_rng(3).normal(
        size=osur._mlp.nparam(16)) * 0.05, np.zeros(16), np.ones(16), 1.0)
    got = osur.query(sc.grid, wf, rf, net, sc.human_xy, sc.radius,
                     sc.height, c, r, s, margin=np.inf, band=0.0,
                     hinge_eps=0.2)
    want = oracle.query(sc.grid, wf, c, r, s, hinge_eps=0.2)
    for a, b in zip(got[:4], want):
        np.testing.assert_array_equal(a, b)
    assert (got[4] == (s >= 0)).all()


def test_nonfinite_network_falls_back():
    sc, rf, wf = room(seed=46, boxes=0)
    c, r, s = queries(sc, seed=4)

    def net(x, k):
        return (np.full(len(x), np.nan, np.float32),
                np.zeros((len(x), 16), np.float32))
    d, _, _, _, used = osur.query(sc.grid, wf, rf, net, sc.human_xy,
                                  sc.radius, sc.height, c, r, s,
                                  margin=0.0, band=0.0)
    ed, _, _, _ = oracle.query(sc.grid, wf, c, r, s)
    # with no environment every in-grid query has a present human (NaN)
    # or none at all (the environment's +inf: not finite): all fall back
    pos = s >= 0
    assert (used[pos] == 1).all()
    np.testing.assert_array_equal(d[pos], ed[pos])


def test_absent_humans_are_ignored_and_clipped_humans_fall_back():
    sc, rf, wf = room(seed=47, K=2)
    h = sc.grid.h
    L = np.array(sc.grid.extent)
    xy = sc.human_xy.copy()
    xy[:, 1] = [L[0] + sc.radius + 2 * h, 0.5 * L[1]]   # wholly outside
    c, r, s = queries(sc, seed=5, lo=0.0, hi=1.0)
    rng = np.random.default_rng(6)
    p = rng.normal(size=osur._mlp.nparam(16)) * 0.02
    net = osur.network(p, np.zeros(16), np.ones(16), 1.0)
    _, wf2 = oracle.predicted_composite(sc.grid, oracle.build_static(
        sc.grid, sc.occ)[0], xy, sc.radius, sc.height)
    a = osur.query(sc.grid, wf2, rf, net, xy, sc.radius, sc.height, c, r, s,
                   margin=0.02, band=0.1)
    b = osur.query(sc.grid, wf2, rf, net, xy[:, :1], sc.radius, sc.height,
                   c, r, s, margin=0.02, band=0.1)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    # a human straddling the grid's edge: clipped, every query it could
    # decide falls back
    xy[:, 1] = [0.05, 0.5 * L[1]]
    _, wf3 = oracle.predicted_composite(sc.grid, oracle.build_static(
        sc.grid, sc.occ)[0], xy, sc.radius, sc.height)
    g, _ = osur.lattice(sc.grid, c)
    G = osur.human_geometry(sc.grid, xy, sc.radius, sc.height, g, s,
                            np.ones(len(s), np.int64))
    assert G["clipped"][s >= 0].all()
    d, _, _, _, used = osur.query(sc.grid, wf3, rf, net, xy, sc.radius,
                                  sc.height, c, r, s, margin=0.02, band=0.1)
    yk, _ = osur.value_and_gradient(G, g, h, *net(osur.features(G, g), 1))
    # no answered query has the clipped human within the band of its
    # answer, and some queries fell back for it
    acc = (used == 0) & (s >= 0)
    assert acc.any()
    assert np.all(yk[acc].astype(np.float64) >
                  (d[acc] + r[acc]).astype(np.float64) + 0.1)
    free = osur.query(sc.grid, wf3, rf, net, xy[:, :1], sc.radius,
                      sc.height, c, r, s, margin=0.02, band=0.1)[4]
    assert np.any((used == 1) & (free == 0) & (s >= 0))

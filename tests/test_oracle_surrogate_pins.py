"""Pins of the surrogate-query oracle (accept / fallback rule) by cases
whose answer is known without it: a constant network (closed form), an
infinite margin (reduces to the exact query), a non-finite network, the
input layout, and the boundary of the span of voxel centres."""
import numpy as np

import oracle
import scenegen
from oracle import mlp as omlp
from oracle import surrogate as osur


def scene():
    sc = scenegen.small_scene(41, 14, 12, 10, h=0.1, n_humans=3, n_slices=3)
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    _, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                       sc.height)
    st = scenegen.human_state(sc.meta["start"], sc.meta["vel"])
    return sc, wf, st


def queries(sc, Q=400, seed=0):
    rng = np.random.default_rng(seed)
    L = np.array(sc.grid.extent)
    c = (rng.uniform(-0.1, 1.1, size=(Q, 3)) * L).astype(np.float32)
    r = rng.uniform(0, 0.3, size=Q).astype(np.float32)
    s = rng.integers(-1, sc.n_slices + 2, size=Q).astype(np.int32)
    return c, r, s


def const_net(value):
    p = np.zeros(omlp.NPARAM)
    p[-1] = value  # output bias: y = value * out_scale everywhere
    return p


def test_constant_network_closed_form():
    sc, wf, st = scene()
    c, r, s = queries(sc)
    ones, zeros = np.ones(22, np.float32), np.zeros(22, np.float32)
    d, g, status, cost, used, _ = osur.query(
        sc.grid, wf, const_net(0.5), zeros, ones, 1.0, st, sc.dt, c, r, s,
        margin=0.1, hinge_eps=0.4)
    ed, eg, est, ecost = oracle.query(sc.grid, wf, c, r, s, hinge_eps=0.4)
    inside = osur.in_span(sc.grid, c)
    accept = inside & (s >= 0) & (np.float32(0.5) - r >= np.float32(0.1))
    assert accept.any() and (~accept & (s >= 0)).any()
    np.testing.assert_array_equal(d[accept], np.float32(0.5) - r[accept])
    np.testing.assert_array_equal(g[accept], 0.0)
    np.testing.assert_array_equal(
        status[accept], np.where(s[accept] > sc.n_slices - 1, 8, 0))
    np.testing.assert_array_equal(
        cost[accept],
        np.maximum(0.4 - (np.float32(0.5) - r[accept]).astype(np.float64),
                   0).astype(np.float32))
    rest = ~accept
    np.testing.assert_array_equal(d[rest], ed[rest])
    np.testing.assert_array_equal(status[rest], est[rest])
    np.testing.assert_array_equal(used, (~accept & (s >= 0)).astype(np.uint8))
    # slice < 0: NaN and the SLICE_NEG bit, never a fallback
    neg = s < 0
    assert np.isnan(d[neg]).all() and (status[neg] == 32).all()


def test_infinite_margin_is_the_exact_query():
    sc, wf, st = scene()
    c, r, s = queries(sc, seed=1)
    p = np.random.default_rng(3).normal(size=omlp.NPARAM) * 0.05
    ones, zeros = np.ones(22, np.float32), np.zeros(22, np.float32)
    got = osur.query(sc.grid, wf, p, zeros, ones, 1.0, st, sc.dt, c, r, s,
                     margin=np.inf, hinge_eps=0.2)
    want = oracle.query(sc.grid, wf, c, r, s, hinge_eps=0.2)
    for a, b in zip(got[:4], want):
        np.testing.assert_array_equal(a, b)
    assert (got[4] == (s >= 0)).all()


def test_nonfinite_network_falls_back():
    sc, wf, st = scene()
    c, r, s = queries(sc, seed=2)
    ones, zeros = np.ones(22, np.float32), np.zeros(22, np.float32)
    got = osur.query(sc.grid, wf, const_net(1.0), zeros, ones, np.inf, st,
                     sc.dt, c, r, s, margin=0.1)
    want = oracle.query(sc.grid, wf, c, r, s)
    np.testing.assert_array_equal(got[0], want[0])
    assert (got[4] == (s >= 0)).all()


def test_feature_layout():
    """A worked example with exact binary values: human 0 starts at (1, 1)
    with velocity (2, -2); at slice 2 of dt = 0.25 (t = 0.5) its axis is at
    (2, 0), so a centre at (5, 4) is 3, 4 from it and 5 from the axis.
    Slices are clamped to [0, n-1] for t."""
    st = np.zeros(18, np.float32)
    st[0:6] = [1, 1, 0, 2, -2, 0]
    st[6:12] = [5, 4, 0, 0, 0, 0]      # on the centre: rho = 0
    st[12:18] = [-1, 4, 0, 0.5, 0, 0]  # axis at (-0.75, 4) at t = 0.5
    c = np.array([[5, 4, 7], [5, 4, 7]], np.float32)
    x = osur.features(c, np.array([2, 9]), 3, 0.25, st)
    np.testing.assert_array_equal(x[0, :4], [5, 4, 7, 0.5])
    np.testing.assert_array_equal(x[0, 4:10], [3, 4, 5, 2, -2, 0])
    np.testing.assert_array_equal(x[0, 10:16], [0, 0, 0, 0, 0, 0])
    np.testing.assert_array_equal(x[0, 16:22], [5.75, 0, 5.75, 0.5, 0, 0])
    assert x[1, 3] == np.float32(2) * np.float32(0.25)  # slice 9 -> n-1 = 2


def test_centre_gradient_unit_cases():
    """dy/dc through the transform for unit feature gradients: the centre
    itself, a human's offsets (+1 along their axis) and its axis distance
    (the unit vector away from the axis, 0 on the axis)."""
    st = np.zeros(18, np.float32)
    st[0:6] = [1, 1, 0, 2, -2, 0]
    st[6:12] = [5, 4, 0, 0, 0, 0]
    x = osur.features(np.array([[5, 4, 7]], np.float32), np.array([2]), 3,
                      0.25, st)
    cases = {0: [1, 0, 0], 1: [0, 1, 0], 2: [0, 0, 1], 3: [0, 0, 0],
             4: [1, 0, 0], 5: [0, 1, 0], 6: [0.6, 0.8, 0], 7: [0, 0, 0],
             12: [0, 0, 0]}  # 12: rho of human 1, who stands on the centre
    for f, want in cases.items():
        G = np.zeros((1, 22))
        G[0, f] = 1.0
        np.testing.assert_allclose(osur.centre_gradient(x, G)[0], want,
                                   rtol=0, atol=1e-7, err_msg=str(f))


def test_centre_gradient_matches_finite_differences():
    """The chain rule against central differences of the fp64 network
    (no rounding) composed with the feature transform, away from the
    humans' axes."""
    rng = np.random.default_rng(5)
    p = omlp.pack([rng.normal(0, 0.3, s) for s in omlp.SHAPES])
    off = np.zeros(22)
    scl = np.full(22, 0.4)
    st = np.zeros(18, np.float32)
    st[0:6] = [1.0, 1.5, 0, 0.5, -0.25, 0]
    st[6:12] = [3.0, 0.5, 0, -0.5, 0.75, 0]
    st[12:18] = [0.5, 3.5, 0, 1.0, 0.0, 0]
    c = np.array([[2.2, 2.9, 1.1], [0.4, 0.9, 0.3], [3.3, 3.1, 1.9]],
                 np.float64)
    s = np.array([1, 3, 2])

    def y_of(cc):
        xx = osur.features(cc.astype(np.float32), s, 5, 0.25, st)
        return omlp.forward(p, xx, off, scl, 1.0, rounding=False)[0]
    x = osur.features(c.astype(np.float32), s, 5, 0.25, st)
    G = omlp.input_gradient(p, x, off, scl, 1.0, rounding=False)
    g = osur.centre_gradient(x, G)
    eps = 1e-2
    for a in range(3):
        d = np.zeros(3)
        d[a] = eps
        num = (y_of(c + d) - y_of(c - d)) / (2 * eps)
        np.testing.assert_allclose(g[:, a], num, rtol=2e-3, atol=2e-4)


def test_span_boundary():
    g = scenegen.Grid(4, 5, 6, 0.5)
    first = np.array([[0.25, 0.25, 0.25]], np.float32)
    last = np.array([[1.75, 2.25, 2.75]], np.float32)
    assert osur.in_span(g, first)[0] and osur.in_span(g, last)[0]
    assert not osur.in_span(g, first - np.float32(1e-3))[0]
    assert not osur.in_span(g, last + np.float32(1e-3))[0]


def test_environment_min_closed_form():
    # Constant network 0.3 with the environment field: the prediction is
    # min(e, 0.3) with e the exact environment value at the centre.
    sc, wf, st = scene()
    rs, rf = oracle.build_static(sc.grid, sc.occ)
    c, r, s = queries(sc, seed=4)
    ones, zeros = np.ones(22, np.float32), np.zeros(22, np.float32)
    d, g, status, cost, used, _ = osur.query(
        sc.grid, wf, const_net(0.3), zeros, ones, 1.0, st, sc.dt, c, r, s,
        margin=0.05, static_sdf=rf)
    e, eg, _, _ = oracle.query(sc.grid, rf[None], c, np.zeros_like(r),
                               np.zeros_like(s))
    v = np.minimum(e, np.float32(0.3))
    inside = osur.in_span(sc.grid, c)
    accept = inside & (s >= 0) & (v - r >= np.float32(0.05))
    assert accept.any() and (accept & (e < 0.3)).any()
    np.testing.assert_array_equal(d[accept], (v - r)[accept])
    env = accept & (e <= np.float32(0.3))
    np.testing.assert_array_equal(g[env], eg[env])
    np.testing.assert_array_equal(g[accept & ~env], 0.0)
    np.testing.assert_array_equal(used, (~accept & (s >= 0)).astype(np.uint8))

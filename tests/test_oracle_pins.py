"""Pins of the CPU oracle against things other than itself.

Brute force from the definition on tiny grids, hand-worked fixtures,
closed forms for boxes, single voxels and voxelised cylinders, the Gauss
circle counts, textbook/library special cases (scipy's linear
interpolation) and invariants of exact EDTs.  None of these retypes the
oracle's separable algorithm.  CPU only.
"""
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
import scenegen
from scenegen import Grid

GOLD = os.path.join(os.path.dirname(__file__), "golden")
INF32 = oracle.INF32
INF64 = oracle.INF64


def brute_edt(mask, want=1):
    """min over voxels u with (mask[u] != 0) == want of |v-u|^2, by
    exhaustive search (int64; INF64 where no such voxel)."""
    nz, ny, nx = mask.shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    allv = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], 1).astype(np.int64)
    sel = (mask.ravel() != 0) == bool(want)
    S = allv[sel]
    if len(S) == 0:
        return np.full(mask.shape, INF64, dtype=np.int64)
    out = np.empty(len(allv), dtype=np.int64)
    for s in range(0, len(allv), 512):
        d = ((allv[s:s + 512, None, :] - S[None, :, :]) ** 2).sum(-1)
        out[s:s + 512] = d.min(1)
    return out.reshape(mask.shape)


def brute_ssq(mask):
    eo = brute_edt(mask, 1)
    ef = brute_edt(mask, 0)
    out = np.where(mask != 0, -np.minimum(ef, INF32),
                   np.minimum(eo, INF32))
    return out.astype(np.int64)


def _masks(rng, shape):
    V = int(np.prod(shape))
    yield np.zeros(shape, np.uint8)
    one = np.zeros(V, np.uint8)
    one[rng.integers(V)] = 1
    yield one.reshape(shape)
    for p in (0.01, 0.1, 0.5, 0.99):
        yield (rng.random(shape) < p).astype(np.uint8)
    yield np.ones(shape, np.uint8)


# ----------------------------------------------------------------- 1-D pass

def test_envelope_1d_matches_direct_min():
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 7, 64, 65, 200):
        for p_inf in (0.0, 0.5, 0.95, 1.0):
            f = rng.integers(0, 3 * 60 ** 2, size=n).astype(np.int64)
            f[rng.random(n) < p_inf] = INF64
            got = oracle.envelope_1d(f)
            q = np.arange(n)
            fin = f != INF64
            if not fin.any():
                assert (got == INF64).all()
                continue
            ref = (f[fin][None, :] + (q[:, None] - q[fin][None, :]) ** 2)
            np.testing.assert_array_equal(got, ref.min(1))


def test_envelope_1d_ties_and_constant():
    # A constant column keeps every site on the envelope.
    f = np.full(50, 7, dtype=np.int64)
    np.testing.assert_array_equal(oracle.envelope_1d(f), f)
    # Equal-value neighbours and a single site.
    f = np.full(9, INF64, dtype=np.int64)
    f[4] = 0
    np.testing.assert_array_equal(oracle.envelope_1d(f),
                                  (np.arange(9) - 4) ** 2)


# --------------------------------------------------------- brute force EDT

@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 9), (1, 7, 1),
                                   (5, 1, 1), (4, 5, 6), (12, 12, 12),
                                   (3, 11, 7), (2, 12, 10)])
def test_edt_and_ssq_match_brute_force(shape):
    rng = np.random.default_rng(sum(shape))
    for m in _masks(rng, shape):
        np.testing.assert_array_equal(oracle.edt_sq(m), brute_edt(m, 1))
        np.testing.assert_array_equal(oracle.signed_sq(m).astype(np.int64),
                                      brute_ssq(m))


def test_hand_worked_2d():
    lines = [l.split() for l in open(os.path.join(GOLD, "ssq_hand_2d.txt"))
             if l.strip() and not l.startswith("#")]
    occ = np.zeros((1, 4, 5), np.uint8)
    for i, j, k in (map(int, l) for l in lines[:2]):
        occ[k, j, i] = 1
    want = np.array([[int(x) for x in l] for l in lines[2:]])
    np.testing.assert_array_equal(oracle.signed_sq(occ)[0], want)


def test_hand_worked_block():
    occ = np.zeros((5, 5, 5), np.uint8)
    occ[1:4, 1:4, 1:4] = 1
    ssq = oracle.signed_sq(occ)
    for l in open(os.path.join(GOLD, "ssq_hand_block.txt")):
        if not l.strip() or l.startswith("#"):
            continue
        i, j, k, v = map(int, l.split())
        assert ssq[k, j, i] == v, (i, j, k)


def test_empty_and_full_sets():
    z = np.zeros((3, 4, 5), np.uint8)
    assert (oracle.signed_sq(z) == INF32).all()
    assert (oracle.signed_sq(1 - z) == -INF32).all()
    assert (oracle.edt_sq(z) == INF64).all()


# ----------------------------------------------------------- closed forms

def box_union_outside(boxes, shape):
    """Squared distance to a union of inclusive index boxes:
    min over boxes of sum_a (v_a - clamp(v_a, lo_a, hi_a))^2."""
    nz, ny, nx = shape
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    best = np.full(shape, INF64, dtype=np.int64)
    for i0, i1, j0, j1, k0, k1 in boxes:
        d = ((ii - np.clip(ii, i0, i1)) ** 2 + (jj - np.clip(jj, j0, j1)) ** 2
             + (kk - np.clip(kk, k0, k1)) ** 2)
        best = np.minimum(best, d)
    return best


@pytest.mark.parametrize("maker", ["cube64", "small"])
def test_box_scenes_outside_closed_form(maker):
    if maker == "cube64":
        sc = scenegen.cube64()
    else:
        sc = scenegen.small_scene(7, 37, 29, 23, h=0.05, n_boxes=9)
    ssq = oracle.signed_sq(sc.occ)
    cf = box_union_outside(sc.boxes, sc.occ.shape)
    free = sc.occ == 0
    np.testing.assert_array_equal(ssq[free].astype(np.int64), cf[free])
    assert (cf[~free] == 0).all()


def test_isolated_box_inside_closed_form():
    shape = (14, 16, 18)
    nz, ny, nx = shape
    lo, hi = (3, 4, 2), (12, 9, 13)   # i, j, k inclusive
    occ = np.zeros(shape, np.uint8)
    occ[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = 1
    ssq = oracle.signed_sq(occ)
    n = (nx, ny, nz)
    for k in range(lo[2], hi[2] + 1):
        for j in range(lo[1], hi[1] + 1):
            for i in range(lo[0], hi[0] + 1):
                v = (i, j, k)
                cands = []
                for a in range(3):
                    if lo[a] - 1 >= 0:
                        cands.append((v[a] - lo[a] + 1) ** 2)
                    if hi[a] + 1 < n[a]:
                        cands.append((hi[a] + 1 - v[a]) ** 2)
                assert ssq[k, j, i] == -min(cands)


def test_box_touching_grid_boundary_inside():
    # A slab filling the whole grid in x and y: the only free voxels are
    # above it, so inside values are -(distance to the top face + 1)^2.
    occ = np.zeros((6, 4, 5), np.uint8)
    occ[:3] = 1
    ssq = oracle.signed_sq(occ)
    for k in range(3):
        assert (ssq[k] == -((3 - k) ** 2)).all()
    for k in range(3, 6):
        assert (ssq[k] == (k - 2) ** 2).all()


def test_single_voxel_closed_form():
    shape = (9, 8, 11)
    occ = np.zeros(shape, np.uint8)
    u = (7, 2, 5)  # i, j, k
    occ[u[2], u[1], u[0]] = 1
    kk, jj, ii = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    want = (ii - u[0]) ** 2 + (jj - u[1]) ** 2 + (kk - u[2]) ** 2
    got = oracle.edt_sq(occ)
    np.testing.assert_array_equal(got, want)


def test_box_continuous_bounds():
    # d_cont <= h*sqrt(E) <= d_cont + sqrt(3) h for voxel centres outside a
    # metric box whose sides are at least h.
    g = Grid(40, 30, 20, 0.05)
    box_m = np.array([[0.52, 1.31, 0.33, 0.91, 0.2, 0.7]])
    idx, occ = scenegen.voxelise_boxes(g, box_m)
    E = oracle.edt_sq(occ)
    kk, jj, ii = np.meshgrid(*[np.arange(s) for s in g.shape_zyx],
                             indexing="ij")
    c = [(ii + 0.5) * g.h, (jj + 0.5) * g.h, (kk + 0.5) * g.h]
    d2 = 0.0
    for a in range(3):
        lo, hi = box_m[0, 2 * a], box_m[0, 2 * a + 1]
        d2 = d2 + (c[a] - np.clip(c[a], lo, hi)) ** 2
    dc = np.sqrt(d2)
    dv = g.h * np.sqrt(E.astype(np.float64))
    free = occ == 0
    assert (dv[free] >= dc[free] - 1e-12).all()
    assert (dv[free] <= dc[free] + math.sqrt(3) * g.h + 1e-12).all()


# -------------------------------------------------- voxelised cylinders

def test_cylinder_layer_counts_gauss_circle():
    g = Grid(25, 25, 8, 0.05)
    for l in open(os.path.join(GOLD, "gauss_circle.txt")):
        if not l.strip() or l.startswith("#"):
            continue
        r, count = map(int, l.split())
        xy = np.array([[12.5 * g.h, 12.5 * g.h]])   # centre of voxel (12,12)
        occ = oracle.human_occupancy(g, xy, r * g.h, 10.0)
        for k in range(g.nz):
            assert int(occ[k].sum()) == count, (r, k)


def test_cylinder_height_layers():
    g = Grid(8, 8, 50, 0.05)
    xy = np.array([[0.2, 0.2]])
    # A voxel layer k is inside iff its centre (k+1/2)h is at most H.
    for H, layers in ((1.8, 36), (0.024, 0), (0.025, 1), (0.076, 2),
                      (10.0, 50)):
        occ = oracle.human_occupancy(g, xy, 0.1, H)
        col = occ[:, 4, 4]
        assert int(col.sum()) == layers, H
        assert (col[:layers] == 1).all()


def _disk_chords(r, ny):
    """Rows of a disk of integer voxel radius r centred on voxel (c, c):
    half-width floor(sqrt(r^2 - dj^2)) by integer square root."""
    return {dj: math.isqrt(r * r - dj * dj) for dj in range(-r, r + 1)}


def test_cylinder_field_closed_form():
    # One cylinder of radius 4 voxels centred on voxel (15, 12), height
    # covering layers 0..9 of 16: exact outside field by the prism formula
    # min over disk rows of (j-j')^2 + (i - clamp(i, a_j', b_j'))^2 plus the
    # z term, and the inside field -min(E_plane_complement, (Kt+1-k)^2).
    g = Grid(31, 26, 16, 0.05)
    ci, cj, r = 15, 12, 4
    H = 10 * g.h
    xy = np.array([[(ci + 0.5) * g.h, (cj + 0.5) * g.h]])
    occ = oracle.human_occupancy(g, xy, r * g.h, H)
    ssq = oracle.signed_sq(occ).astype(np.int64)
    Kt = 9
    ch = _disk_chords(r, g.ny)
    plane = np.zeros((g.ny, g.nx), np.uint8)
    for dj, w in ch.items():
        plane[cj + dj, ci - w:ci + w + 1] = 1
    assert (occ[:Kt + 1] == plane[None]).all()
    assert (occ[Kt + 1:] == 0).all()
    # 2-D complement distance by brute force on the plane only.
    ein2 = brute_edt(plane[None], 0)[0]
    for k in range(g.nz):
        dz = max(0, k - Kt)
        for j in range(g.ny):
            for i in range(g.nx):
                if occ[k, j, i]:
                    want = -min(int(ein2[j, i]), (Kt + 1 - k) ** 2)
                else:
                    best = min((j - (cj + dj)) ** 2 +
                               (i - min(max(i, ci - w), ci + w)) ** 2
                               for dj, w in ch.items())
                    want = best + dz * dz
                assert ssq[k, j, i] == want, (i, j, k)


def test_cylinders_outside_grid_are_clipped():
    g = Grid(20, 20, 10, 0.05)
    far = np.array([[-5.0, 0.3], [0.3, 7.0]])
    assert oracle.human_occupancy(g, far, 0.25, 1.8).sum() == 0
    part = np.array([[-0.1, 0.5]])   # straddles x = 0
    occ = oracle.human_occupancy(g, part, 0.25, 1.8)
    assert 0 < occ.sum() < 10 * math.pi * 25


def test_cylinder_rejects_non_finite():
    g = Grid(4, 4, 4, 0.05)
    with pytest.raises(ValueError):
        oracle.human_occupancy(g, np.array([[np.nan, 0.0]]), 0.25, 1.8)


# ------------------------------------------------------------- invariants

def _scene_small(seed=3):
    return scenegen.small_scene(seed, 33, 27, 21, h=0.05, n_boxes=7,
                                n_humans=3, n_slices=4)


def test_I1_I7_composite_outside_is_union_edt_and_sign_is_union():
    sc = _scene_small()
    ssq_s, _ = oracle.build_static(sc.grid, sc.occ)
    c, _ = oracle.predicted_composite(sc.grid, ssq_s, sc.human_xy,
                                      sc.radius, sc.height)
    for s in range(sc.n_slices):
        hocc = oracle.human_occupancy(sc.grid, sc.human_xy[s], sc.radius,
                                      sc.height)
        union = ((sc.occ != 0) | (hocc != 0)).astype(np.uint8)
        eu = brute_edt(union, 1) if union.size <= 20000 else \
            oracle.edt_sq(union)
        cs = c[s].astype(np.int64)
        np.testing.assert_array_equal(np.maximum(cs, 0),
                                      np.where(union != 0, 0, eu))
        np.testing.assert_array_equal(cs < 0, union != 0)      # I7


def test_I1_by_brute_force_tiny():
    sc = scenegen.small_scene(5, 12, 11, 10, h=0.1, n_boxes=3, n_humans=2,
                              n_slices=2, radius=0.2, height=0.6)
    ssq_s, _ = oracle.build_static(sc.grid, sc.occ)
    c, _ = oracle.predicted_composite(sc.grid, ssq_s, sc.human_xy,
                                      sc.radius, sc.height)
    for s in range(sc.n_slices):
        hocc = oracle.human_occupancy(sc.grid, sc.human_xy[s], sc.radius,
                                      sc.height)
        union = ((sc.occ != 0) | (hocc != 0)).astype(np.uint8)
        eu = brute_edt(union, 1)
        cs = c[s].astype(np.int64)
        np.testing.assert_array_equal(np.maximum(cs, 0),
                                      np.where(union != 0, 0, eu))
        # inside: min of the two signed fields, each by brute force
        hs = brute_ssq(hocc)
        ss = brute_ssq(sc.occ)
        np.testing.assert_array_equal(cs, np.minimum(ss, hs))


def test_I2_pass_order():
    rng = np.random.default_rng(5)
    m = (rng.random((9, 13, 11)) < 0.07).astype(np.uint8)
    ref = oracle.edt_sq_order(m, (0, 1, 2))
    for order in ((2, 1, 0), (1, 2, 0), (1, 0, 2), (2, 0, 1)):
        np.testing.assert_array_equal(oracle.edt_sq_order(m, order), ref)


def test_I3_flip_and_permutation_equivariance():
    rng = np.random.default_rng(8)
    m = (rng.random((10, 12, 14)) < 0.05).astype(np.uint8)
    ref = oracle.signed_sq(m)
    for ax in range(3):
        np.testing.assert_array_equal(oracle.signed_sq(np.flip(m, ax)),
                                      np.flip(ref, ax))
    mc = (rng.random((9, 9, 9)) < 0.1).astype(np.uint8)
    rc = oracle.signed_sq(mc)
    for perm in ((1, 0, 2), (2, 1, 0), (0, 2, 1)):
        np.testing.assert_array_equal(
            oracle.signed_sq(np.transpose(mc, perm)), np.transpose(rc, perm))


def test_I4_translation():
    m = np.zeros((12, 14, 16), np.uint8)
    m[3:5, 4:7, 2:4] = 1
    m[7, 9, 10] = 1
    ref = oracle.edt_sq(m)
    sh = np.roll(m, (2, -1, 3), axis=(0, 1, 2))
    got = oracle.edt_sq(sh)
    # Away from the wrapped border the field must move with the set only
    # when no far-away site is cut off; compare on the full grid by
    # embedding both in a larger padded grid instead.
    big = np.zeros((20, 22, 24), np.uint8)
    big[4:16, 4:18, 4:20] = m
    big2 = np.zeros_like(big)
    big2[6:18, 3:17, 7:23] = m
    e1 = oracle.edt_sq(big)
    e2 = oracle.edt_sq(big2)
    np.testing.assert_array_equal(e1[4:14, 4:16, 4:20],
                                  e2[6:16, 3:15, 7:23])
    assert got.shape == ref.shape


def test_I5_lipschitz_and_I6_zero_set():
    rng = np.random.default_rng(9)
    m = (rng.random((15, 16, 17)) < 0.03).astype(np.uint8)
    e = np.sqrt(oracle.edt_sq(m).astype(np.float64))
    for ax in range(3):
        d = np.abs(np.diff(e, axis=ax))
        assert (d <= 1.0 + 1e-12).all()
    np.testing.assert_array_equal(oracle.edt_sq(m) == 0, m != 0)


def test_I8_F_commutes_with_min_and_F_values():
    rng = np.random.default_rng(4)
    a = rng.integers(-3 * 512 ** 2, 3 * 512 ** 2, size=5000).astype(np.int32)
    b = rng.integers(-3 * 512 ** 2, 3 * 512 ** 2, size=5000).astype(np.int32)
    a[:3] = [INF32, -INF32, 1]
    h = 0.02
    np.testing.assert_array_equal(
        oracle.to_float(np.minimum(a, b), h),
        np.minimum(oracle.to_float(a, h), oracle.to_float(b, h)))
    # perfect squares give exact multiples of (float)h
    sq = np.array([1, 4, 9, 16, 10000, -25], dtype=np.int32)
    want = np.float32(h) * np.array([1, 2, 3, 4, 100, -5], dtype=np.float32)
    np.testing.assert_array_equal(oracle.to_float(sq, h), want)
    # against a correctly rounded numpy sqrt in float32
    x = rng.integers(1, 3 * 1023 ** 2, size=20000).astype(np.int32)
    ref = np.float32(h) * np.sqrt(x.astype(np.float32))
    np.testing.assert_array_equal(oracle.to_float(x, h), ref)
    assert np.isposinf(oracle.to_float(np.array([INF32], np.int32), h)[0])
    assert np.isneginf(oracle.to_float(np.array([-INF32], np.int32), h)[0])


def test_I9_cartesian_product():
    # A vertical prism A x B: E = E_A(x, y) + E_B(z).
    rng = np.random.default_rng(21)
    A = (rng.random((13, 17)) < 0.1).astype(np.uint8)
    B = np.zeros(11, np.uint8)
    B[3:6] = 1
    m = (B[:, None, None] * A[None]).astype(np.uint8)
    eA = brute_edt(A[None], 1)[0]
    eB = brute_edt(B[:, None, None], 1)[:, 0, 0]
    np.testing.assert_array_equal(oracle.edt_sq(m),
                                  eB[:, None, None] + eA[None])


def test_I10_no_humans_in_grid_gives_static():
    sc = _scene_small(4)
    ssq_s, sdf_s = oracle.build_static(sc.grid, sc.occ)
    far = np.full_like(sc.human_xy, -50.0)
    c, cf = oracle.predicted_composite(sc.grid, ssq_s, far, sc.radius,
                                       sc.height)
    for s in range(sc.n_slices):
        np.testing.assert_array_equal(c[s], ssq_s)
        np.testing.assert_array_equal(cf[s], sdf_s)


# ---------------------------------------------------------------- queries

def _planar(g, n_slices=2):
    kk, jj, ii = np.meshgrid(*[np.arange(s) for s in g.shape_zyx],
                             indexing="ij")
    a, b, c, d = 0.6, -0.3, 0.74, 0.125
    x = (ii + 0.5) * g.h
    y = (jj + 0.5) * g.h
    z = (kk + 0.5) * g.h
    f = (a * x + b * y + c * z + d).astype(np.float32)
    return np.stack([f + s for s in range(n_slices)]), (a, b, c, d)


def test_I13_planar_field_exact_and_constant_gradient():
    g = Grid(10, 12, 9, 0.05)
    field, (a, b, c, d) = _planar(g)
    rng = np.random.default_rng(1)
    Q = 500
    lo, hi = g.h / 2, np.array(g.extent) - g.h / 2
    cen = (rng.random((Q, 3)) * (hi - lo) + lo).astype(np.float32)
    r = rng.uniform(0.05, 0.15, Q).astype(np.float32)
    s = (np.arange(Q) % 2).astype(np.int32)
    dist, grad, st, _ = oracle.query(g, field, cen, r, s)
    cd = cen.astype(np.float64)
    want = a * cd[:, 0] + b * cd[:, 1] + c * cd[:, 2] + d + s - r
    np.testing.assert_allclose(dist, want, rtol=0, atol=2e-6)
    np.testing.assert_allclose(grad, np.tile([a, b, c], (Q, 1)), atol=2e-5)
    assert (st == 0).all()


def test_query_matches_scipy_linear_interpolation_and_fd_gradient():
    sc = _scene_small(6)
    g = sc.grid
    ssq_s, sdf_s = oracle.build_static(g, sc.occ)
    rng = np.random.default_rng(3)
    Q = 400
    lo, hi = g.h / 2, np.array(g.extent) - g.h / 2
    cen = (rng.random((Q, 3)) * (hi - lo) + lo).astype(np.float32)
    r = np.zeros(Q, np.float32)
    s = np.zeros(Q, np.int32)
    dist, grad, st, _ = oracle.query(g, sdf_s[None], cen, r, s)
    gc = (cen.astype(np.float64) / g.h - 0.5)
    ref = ndimage.map_coordinates(sdf_s.astype(np.float64),
                                  [gc[:, 2], gc[:, 1], gc[:, 0]], order=1,
                                  mode="nearest")
    np.testing.assert_allclose(dist, ref, rtol=1e-6, atol=1e-6)
    # gradient = central difference of the interpolant inside the same cell
    eps = 1e-4
    for a in range(3):
        cp = gc.copy()
        cm = gc.copy()
        fl = np.floor(gc[:, a])
        cp[:, a] = np.minimum(gc[:, a] + eps, fl + 1 - 1e-9)
        cm[:, a] = np.maximum(gc[:, a] - eps, fl + 1e-9)
        fp = ndimage.map_coordinates(sdf_s.astype(np.float64),
                                     [cp[:, 2], cp[:, 1], cp[:, 0]], order=1)
        fm = ndimage.map_coordinates(sdf_s.astype(np.float64),
                                     [cm[:, 2], cm[:, 1], cm[:, 0]], order=1)
        fd = (fp - fm) / ((cp[:, a] - cm[:, a]) * g.h)
        np.testing.assert_allclose(grad[:, a], fd, rtol=1e-5, atol=1e-4)


def test_I12_query_at_voxel_centre_returns_stored_value():
    # h = 1/16 m makes voxel centres exact in float32
    sc = scenegen.small_scene(2, 33, 27, 21, h=0.0625, n_boxes=7)
    g = sc.grid
    _, sdf_s = oracle.build_static(g, sc.occ)
    rng = np.random.default_rng(2)
    ijk = np.stack([rng.integers(0, g.nx, 200), rng.integers(0, g.ny, 200),
                    rng.integers(0, g.nz, 200)], 1)
    cen = ((ijk + 0.5) * g.h).astype(np.float32)
    # keep only centres whose float32 coordinate maps back exactly
    gc = cen.astype(np.float64) / g.h - 0.5
    ok = (np.abs(gc - ijk) < 1e-9).all(1)
    dist, _, st, _ = oracle.query(g, sdf_s[None], cen[ok],
                                  np.zeros(ok.sum(), np.float32),
                                  np.zeros(ok.sum(), np.int32))
    want = sdf_s[ijk[ok, 2], ijk[ok, 1], ijk[ok, 0]]
    np.testing.assert_array_equal(dist, want)
    assert ok.sum() == 200


def test_I14_slice_clamp_negative_slice_oor_and_inf():
    g = Grid(6, 5, 4, 0.1)
    field, _ = _planar(g, 3)
    cen = np.array([[0.3, 0.2, 0.2]] * 4 + [[-1.0, 0.2, 9.0]],
                   dtype=np.float32)
    r = np.zeros(5, np.float32)
    s = np.array([2, 3, 99, -1, 0], np.int32)
    dist, grad, st, cost = oracle.query(g, field, cen, r, s, hinge_eps=0.4)
    assert dist[1] == dist[0] and dist[2] == dist[0]
    assert st[0] == 0 and st[1] == oracle.SLICE_CLAMPED
    assert st[2] == oracle.SLICE_CLAMPED
    assert st[3] == oracle.SLICE_NEG and np.isnan(dist[3])
    assert np.isnan(grad[3]).all() and np.isnan(cost[3])
    assert st[4] == oracle.OOR_X | oracle.OOR_Z
    # clamped query equals the query at the clamped point
    d2, _, _, _ = oracle.query(g, field,
                               np.array([[0.05, 0.2, 0.35]], np.float32),
                               np.zeros(1, np.float32),
                               np.zeros(1, np.int32))
    np.testing.assert_allclose(dist[4], d2[0], atol=1e-6)
    assert cost[0] == max(0.0, 0.4 - dist[0]) or \
        abs(cost[0] - max(0.0, 0.4 - float(dist[0]))) < 1e-6
    inf = np.full((1,) + g.shape_zyx, np.inf, np.float32)
    d3, g3, s3, c3 = oracle.query(g, inf, cen[:1], r[:1],
                                  np.zeros(1, np.int32), hinge_eps=0.4)
    assert np.isposinf(d3[0]) and (g3 == 0).all() and \
        s3[0] == oracle.INF_CORNER and c3[0] == 0

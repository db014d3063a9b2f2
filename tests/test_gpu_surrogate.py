"""The per-human surrogate on the GPU (through the C-ABI) against its
oracle.

Rows: pcsdf_surrogate_human_features against oracle/surrogate.py's
features, base distance and residual target (fp64 on both sides, rounded
to fp32; the trig features may differ by the last fp64 bit of sin/cos,
i.e. by at most one fp32 ulp after rounding).

Queries: pcsdf_query_spheres_surrogate against oracle.surrogate.query
with the same network values.  The network itself is held to its own
parity bounds by the MLP tests; here the oracle is given the GPU network's
value and input gradient for every (query, human) row (the fused
inference computes each row on its own, so the values inside the
surrogate call are the same bits), which makes the comparison exact:
identical accept / fallback decisions, bit-identical distances, status
bits and costs, gradients within 1e-6 relative (the chain rule's fp64
sums are ordered differently), and the exact answers of the fallback
queries held to the exact-query contract.
"""
import sys

import numpy as np
import pytest

import oracle
import scenegen
from oracle import mlp as omlp
from oracle import surrogate as osur

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sg(dev):
    import paper_2201_05058_amd.surrogate as m
    return m


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rand_net(seed, gain=1.5, n_in=16):
    r = np.random.default_rng(seed)
    out = []
    for s in omlp.shapes(n_in):
        fan = s[-1] if len(s) == 2 else 16
        out.append(r.uniform(-1, 1, size=s) * gain / np.sqrt(fan))
    p = omlp.pack(out)
    p[-1] = 0.4  # output bias: residuals around the exact field's range
    return p.astype(np.float32)


def make_case(seed, Q=4000, nx=40, ny=36, nz=30, n_slices=4, K=3, h=0.05,
              boxes=6):
    sc = scenegen.small_scene(seed, nx, ny, nz, h=h, n_humans=K,
                              n_slices=n_slices, n_boxes=boxes,
                              radius=0.2, height=0.8)
    rng = np.random.default_rng(seed + 1)
    L = np.array(sc.grid.extent)
    c = (rng.uniform(-0.05, 1.05, size=(Q, 3)) * L).astype(np.float32)
    r = rng.uniform(0, 0.12, size=Q).astype(np.float32)
    s = rng.integers(-1, n_slices + 2, size=Q).astype(np.int32)
    return sc, c, r, s


def norm16(seed):
    r = np.random.default_rng(seed)
    off = (r.normal(size=16) * 0.2).astype(np.float32)
    scl = (0.05 + 0.1 * r.random(16)).astype(np.float32)
    scl[6:] = 1.0  # the trig features are already O(1)
    return off, scl


@pytest.mark.parametrize("seed", [0, 1])
def test_rows_match_oracle(sg, dev, seed):
    sc, c, r, s = make_case(20 + seed, Q=3000)
    K = sc.n_humans
    k = np.random.default_rng(seed).integers(0, K, size=len(s)).astype(
        np.int32)
    g, _ = osur.lattice(sc.grid, c)
    G = osur.human_geometry(sc.grid, sc.human_xy, sc.radius, sc.height, g,
                            s, k)
    wx = osur.features(G, g)
    lab = np.random.default_rng(seed + 7).uniform(0, 2, len(s)).astype(
        np.float32)
    say(f"surrogate rows seed={seed}")
    x, base, tgt = sg.surrogate_human_features(
        sc.grid, sc.human_xy, sc.radius, sc.height, to_dev(c, dev),
        to_dev(s, dev), human=to_dev(k, dev), label=to_dev(lab, dev))
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    # every feature equal, the trig ones within one fp32 ulp
    np.testing.assert_array_equal(x[:, :6], wx[:, :6])
    np.testing.assert_allclose(x[:, 6:], wx[:, 6:], rtol=0, atol=6e-8)
    np.testing.assert_array_equal(base.cpu().numpy(),
                                  G["d"].astype(np.float32))
    want = (lab.astype(np.float64) / sc.grid.h - G["d"]).astype(np.float32)
    np.testing.assert_array_equal(tgt.cpu().numpy(), want)


def gpu_network(sg, net, sc, c, s, dev):
    """(x, k) -> the GPU network's value and input gradient for human k's
    rows of every query (the rows the oracle asks for)."""
    cache = {}

    def run(x, k):
        if k not in cache:
            kk = np.full(len(s), k, np.int32)
            xd, _, _ = sg.surrogate_human_features(
                sc.grid, sc.human_xy, sc.radius, sc.height, to_dev(c, dev),
                to_dev(s, dev), human=to_dev(kk, dev))
            y, gx = net.forward(xd)
            torch.cuda.synchronize()
            cache[k] = (y.cpu().numpy(), gx.cpu().numpy())
        return cache[k]
    return run


CASES = [
    # seed, Q, nx, ny, nz, slices, humans, voxel, boxes, margin, band
    (30, 4000, 40, 36, 30, 4, 3, 0.05, 6, 0.05, 0.17),
    (31, 5000, 57, 33, 21, 3, 5, 0.04, 8, 0.02, 0.0),
    (32, 3000, 48, 48, 16, 2, 1, 0.05, 0, 0.10, 0.10),
    (33, 3000, 33, 41, 19, 5, 0, 0.05, 5, 0.05, 0.17),
]


@pytest.mark.parametrize("case", CASES)
def test_queries_match_oracle(sg, dev, case):
    seed, Q, nx, ny, nz, n, K, h, boxes, margin, band = case
    sc, c, r, s = make_case(seed, Q, nx, ny, nz, n, max(K, 1), h, boxes)
    if K == 0:
        sc.human_xy = np.zeros((n, 0, 2))
    g = sc.grid
    rs, rf = oracle.build_static(g, sc.occ)
    _, wf = oracle.predicted_composite(g, rs, sc.human_xy, sc.radius,
                                       sc.height)
    import paper_2201_05058_amd as pc
    net = sg.Mlp(n_in=16)
    off, scl = norm16(seed)
    net.set_params(rand_net(seed), off, scl, 1.0)
    occ = to_dev(sc.occ, dev)
    ssq, sdf = pc.build_static_sdf(g, occ)
    say(f"surrogate queries {case}")
    out = sg.query_spheres_surrogate(
        net, g, ssq, sdf, sc.human_xy, sc.radius, sc.height, to_dev(c, dev),
        to_dev(r, dev), to_dev(s, dev), fallback_margin=margin, band=band,
        hinge_eps=0.3, want_cost=True)
    torch.cuda.synchronize()
    d = out["dist"].cpu().numpy()
    gr = out["grad"].cpu().numpy()
    st = out["status"].cpu().numpy()
    cost = out["cost"].cpu().numpy()
    used = out["used_fallback"].cpu().numpy()
    wd, wg, wst, wcost, wused = osur.query(
        g, wf, rf, gpu_network(sg, net, sc, c, s, dev), sc.human_xy,
        sc.radius, sc.height, c, r, s, margin=margin, band=band,
        hinge_eps=0.3)
    np.testing.assert_array_equal(used, wused)
    acc = (wused == 0) & (s >= 0)
    ex = wused == 1
    say(f"  answered {acc.mean():.3f} fallback {ex.mean():.3f}")
    if K > 0 and band == 0.0:
        assert acc.mean() > 0.05
    np.testing.assert_array_equal(d[acc], wd[acc])
    np.testing.assert_array_equal(st, wst)
    np.testing.assert_array_equal(cost[acc], wcost[acc])
    assert np.all(np.abs(gr[acc] - wg[acc]) <=
                  1e-6 * np.maximum(np.abs(wg[acc]), 1.0))
    # exact answers: the exact-query contract
    assert np.all(np.abs(d[ex] - wd[ex]) <=
                  1e-6 * np.maximum(np.abs(wd[ex]), g.h))
    assert np.all(np.abs(gr[ex] - wg[ex]) <=
                  1e-6 * np.maximum(np.abs(wg[ex]), 1.0))
    neg = s < 0
    assert np.isnan(d[neg]).all() and (used[neg] == 0).all()
    net.close()


def test_network_of_another_handle_or_width_is_rejected(sg, dev):
    import ctypes as C

    import paper_2201_05058_amd as pc
    from paper_2201_05058_amd import _native
    sc, c, r, s = make_case(40, Q=16)
    g = _native.as_grid(sc.grid)
    occ = to_dev(sc.occ, dev)
    ssq, sdf = pc.build_static_sdf(sc.grid, occ)
    h = pc.default_handle()
    other = pc.Handle()
    xy = np.ascontiguousarray(sc.human_xy, np.float64)
    cd, rd, sd = to_dev(c, dev), to_dev(r, dev), to_dev(s, dev)
    out = torch.empty(16, dtype=torch.float32, device=dev)
    gout = torch.empty((16, 3), dtype=torch.float32, device=dev)

    def call(net):
        return h.lib.pcsdf_query_spheres_surrogate(
            h.ptr, net.ptr, C.byref(g), C.c_void_p(ssq.data_ptr()),
            C.c_void_p(sdf.data_ptr()), xy.shape[0], xy.shape[1],
            xy.ctypes.data_as(C.c_void_p), sc.radius, sc.height, 0.1, 0.0,
            16, C.c_void_p(cd.data_ptr()), C.c_void_p(rd.data_ptr()),
            C.c_void_p(sd.data_ptr()), 0.0, C.c_void_p(out.data_ptr()),
            C.c_void_p(gout.data_ptr()), None, None, None, None, None)
    foreign = sg.Mlp(other, n_in=16)
    foreign.set_params(rand_net(1), *norm16(1), 1.0)
    assert call(foreign) == 1
    assert b"another handle" in h.lib.pcsdf_last_error(h.ptr)
    wide = sg.Mlp(n_in=22)
    wide.set_params(rand_net(2, n_in=22), np.zeros(22), np.ones(22), 1.0)
    assert call(wide) == 1
    assert b"16 inputs" in h.lib.pcsdf_last_error(h.ptr)
    foreign.close()
    wide.close()
    other.close()

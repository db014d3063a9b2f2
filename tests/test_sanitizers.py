"""Host code under the address and undefined-behaviour sanitizers (CPU
only): the C oracle, driven through tests/cpu_device/oracle_driver.c, and
the library's planar-field helpers and batch planner/workers compiled for
the host (tests/cpu_device/harness.cpp).  Each sanitized build runs a
small ragged workload; any report aborts it with a non-zero status, and
its outputs must equal those of the plain builds."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import scenegen
from test_cpu_device_code import HERE, ROOT, SRC, ragged, run_planes

SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer", "-g", "-static-libasan"]
ENV = dict(os.environ, ASAN_OPTIONS="verify_asan_link_order=0:detect_leaks=1",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, timeout=300):
    r = subprocess.run(cmd, capture_output=True, text=True, env=ENV,
                       timeout=timeout)
    assert r.returncode == 0, (r.returncode, r.stderr[-4000:])
    return r


@pytest.fixture(scope="module")
def oracle_san(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "oracle_driver")
    subprocess.run(["gcc", "-O1", "-std=c11", "-ffp-contract=off", *SAN,
                    "-o", exe, os.path.join(HERE, "cpu_device",
                                            "oracle_driver.c"),
                    os.path.join(ROOT, "oracle", "pcsdf_oracle.c"), "-lm"],
                   check=True)
    return exe


@pytest.fixture(scope="module")
def harness_san(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "harness")
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", *SAN,
                    "-I" + os.path.join(HERE, "cpu_device"),
                    "-I" + os.path.join(ROOT, "include"), "-o", exe, SRC],
                   check=True)
    return exe


@pytest.mark.parametrize("dims,K", [((23, 17, 11), 2), ((8, 40, 5), 3),
                                    ((1, 9, 7), 1), ((16, 16, 16), 0)])
def test_oracle_under_sanitizers(oracle_san, tmp_path, dims, K):
    nx, ny, nz = dims
    sc = scenegen.small_scene(60 + nx, nx, ny, nz, h=0.05, n_boxes=3,
                              n_humans=max(K, 1), n_slices=3, n_queries=200)
    xy = sc.human_xy if K else np.zeros((3, 0, 2))
    q = sc.queries
    g = sc.grid
    inp, out = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([nx, ny, nz, 3, K, len(q.radius)], np.int32)
                .tobytes())
        f.write(np.array([g.h, *g.origin, sc.radius, sc.height], np.float64)
                .tobytes())
        f.write(np.ascontiguousarray(sc.occ, np.uint8).tobytes())
        f.write(np.ascontiguousarray(xy, np.float64).tobytes())
        f.write(np.ascontiguousarray(q.centre, np.float32).tobytes())
        f.write(np.ascontiguousarray(q.radius, np.float32).tobytes())
        f.write(np.ascontiguousarray(q.slice, np.int32).tobytes())
    _run([oracle_san, str(inp), str(out)])
    raw = out.read_bytes()
    V, n, Q = g.nvox, 3, len(q.radius)
    o = 0

    def take(dt, cnt):
        nonlocal o
        a = np.frombuffer(raw, dt, cnt, o)
        o += a.nbytes
        return a
    st, c, cf = take(np.int32, V), take(np.int32, n * V), take(np.float32,
                                                                 n * V)
    dist, grad, cost = take(np.float32, Q), take(np.float32, 3 * Q), \
        take(np.float32, Q)
    status = take(np.uint8, Q)
    assert o == len(raw)
    rs, _ = oracle.build_static(g, sc.occ)
    wc, wf = oracle.predicted_composite(g, rs, xy, sc.radius, sc.height)
    wd, wg, wst, wcost = oracle.query(g, wf, q.centre, q.radius, q.slice,
                                      hinge_eps=0.3)
    np.testing.assert_array_equal(st, rs.reshape(-1))
    np.testing.assert_array_equal(c, wc.reshape(-1))
    np.testing.assert_array_equal(cf.view(np.int32), wf.reshape(-1)
                                  .view(np.int32))
    np.testing.assert_array_equal(dist.view(np.int32), wd.view(np.int32))
    np.testing.assert_array_equal(grad.view(np.int32),
                                  wg.reshape(-1).view(np.int32))
    np.testing.assert_array_equal(cost.view(np.int32), wcost.view(np.int32))
    np.testing.assert_array_equal(status, wst)


def test_planar_helpers_under_sanitizers(harness_san, tmp_path):
    for q, (nx, ny, K, r) in enumerate([(37, 29, 2, 0.25), (21, 60, 1, 0.25),
                                        (40, 40, 3, 3.0), (33, 27, 3, 0.0)]):
        sc = scenegen.small_scene(40 + q, nx, ny, 4, h=0.05, n_humans=K,
                                  n_slices=3, radius=r)
        P = run_planes(harness_san, tmp_path, sc)
        g2 = scenegen.Grid(nx, ny, 1, sc.grid.h, sc.grid.origin)
        for s in range(sc.n_slices):
            occ = oracle.human_occupancy(g2, sc.human_xy[s], sc.radius, 10.0)
            np.testing.assert_array_equal(P[s], oracle.signed_sq(occ)[0])


def test_batch_workers_under_sanitizers(harness_san, tmp_path):
    scs = ragged(91)[:5]
    inp, out = str(tmp_path / "b.bin"), str(tmp_path / "b.out")
    stats = []
    with open(inp, "wb") as f:
        f.write(np.array([len(scs), 4, 0, 2, 256, 1], np.int32).tobytes())
        for sc in scs:
            g = sc.grid
            n, K = sc.human_xy.shape[:2]
            rs, _ = oracle.build_static(g, sc.occ)
            stats.append(rs)
            f.write(np.array([g.nx, g.ny, g.nz, n, K], np.int32).tobytes())
            f.write(np.array([g.h, *g.origin, sc.radius, sc.height],
                             np.float64).tobytes())
            f.write(np.ascontiguousarray(sc.human_xy, np.float64).tobytes())
            f.write(np.ascontiguousarray(rs, np.int32).tobytes())
    _run([harness_san, "batch", inp, out])
    res = np.fromfile(out, dtype=np.int32)
    off = 0
    for sc, rs in zip(scs, stats):
        g = sc.grid
        n, V = sc.n_slices, g.nvox
        c = res[off:off + n * V].reshape((n,) + g.shape_zyx)
        off += 2 * n * V
        wc, _ = oracle.predicted_composite(g, rs, sc.human_xy, sc.radius,
                                           sc.height)
        np.testing.assert_array_equal(c, wc)

"""The library's device code compiled for the host and checked against the
oracle, without a GPU.

tests/cpu_device/harness.cpp includes the library's planar-field helpers
and batch planner/workers (with a small stand-in for the HIP names they
use) and is built with g++.  Its planes are compared with the oracle's
signed EDT of the voxelised disks, and its batched composites with the
oracle's per-slice composite, element by element.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import scenegen
from scenegen import Grid

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_device", "harness.cpp")
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("cpu_device") / "harness")
    cmd = ["g++", "-O1", "-std=c++17", "-pthread",
           "-I" + os.path.join(HERE, "cpu_device"),
           "-I" + os.path.join(ROOT, "include"), "-o", exe, SRC]
    subprocess.run(cmd, check=True)
    return exe


def fixed(p, o, h):
    return int(np.rint((p - o) / h * 65536.0))


def run_planes(exe, tmp, sc):
    g = sc.grid
    n, K = sc.human_xy.shape[:2]
    R = fixed(sc.radius, 0.0, g.h)
    xy = [fixed(sc.human_xy[s, k, a], g.origin[a], g.h)
          for s in range(n) for k in range(K) for a in range(2)]
    inp, out = str(tmp / "p.bin"), str(tmp / "p.out")
    with open(inp, "wb") as f:
        f.write(np.array([g.nx, g.ny, n, K], np.int32).tobytes())
        f.write(np.int64(R).tobytes())
        f.write(np.array(xy, np.int64).tobytes())
    subprocess.run([exe, "planes", inp, out], check=True, timeout=120)
    return np.fromfile(out, dtype=np.int32).reshape(n, g.ny, g.nx)


def plane_scenes():
    yield scenegen.room256()
    for q, (nx, ny, K, r) in enumerate([(37, 29, 2, 0.25), (21, 60, 1, 0.25),
                                        (100, 36, 4, 0.25), (64, 64, 8, 0.4),
                                        (40, 40, 3, 3.0), (33, 27, 3, 0.0)]):
        yield scenegen.small_scene(40 + q, nx, ny, 4, h=0.05, n_humans=K,
                                   n_slices=3, radius=r)


@pytest.mark.parametrize("idx", range(7))
def test_planar_helpers_match_oracle(harness, tmp_path, idx):
    sc = list(plane_scenes())[idx]
    P = run_planes(harness, tmp_path, sc)
    g2 = Grid(sc.grid.nx, sc.grid.ny, 1, sc.grid.h, sc.grid.origin)
    for s in range(sc.n_slices):
        occ = oracle.human_occupancy(g2, sc.human_xy[s], sc.radius, 10.0)
        np.testing.assert_array_equal(P[s], oracle.signed_sq(occ)[0])


def ragged(seed):
    # nx*ny odd, divisible by 4 (also with nx odd), 2 mod 4, and odd with
    # V divisible by 4: the composite's 1-, 4- and 2-voxel packs, and 4-wide
    # packs whose planar values are gathered
    dims = [(37, 29, 23, 3, 2), (64, 48, 40, 5, 3), (21, 60, 17, 1, 1),
            (100, 36, 30, 7, 4), (8, 8, 8, 2, 0), (44, 44, 44, 6, 4),
            (34, 27, 13, 3, 2), (33, 27, 20, 2, 2),
            (30, 1000, 6, 2, 8)]  # chord table beyond the items' LDS
    out = []
    for q, (nx, ny, nz, n, K) in enumerate(dims):
        sc = scenegen.small_scene(seed + q, nx, ny, nz, h=0.05, n_boxes=5,
                                  n_humans=max(K, 1), n_slices=n)
        if K == 0:
            sc.human_xy = np.zeros((n, 0, 2))
        out.append(sc)
    return out


@pytest.mark.parametrize("threads,tune", [(8, (0, 0, 0, 0)),
                                          (3, (0, 3, 512, 2)),
                                          (16, (0, 1, 256, 1))])
def test_batch_planner_and_workers_match_oracle(harness, tmp_path, threads,
                                                tune):
    scs = ragged(7 * threads)
    inp, out = str(tmp_path / "b.bin"), str(tmp_path / "b.out")
    stats = []
    with open(inp, "wb") as f:
        f.write(np.array([len(scs), threads, *tune], np.int32).tobytes())
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
    subprocess.run([harness, "batch", inp, out], check=True, timeout=300)
    res = np.fromfile(out, dtype=np.int32)
    off = 0
    for sc, rs in zip(scs, stats):
        g = sc.grid
        n, V = sc.n_slices, g.nvox
        c = res[off:off + n * V].reshape((n,) + g.shape_zyx)
        off += n * V
        f = res[off:off + n * V].reshape((n,) + g.shape_zyx)
        off += n * V
        wc, wf = oracle.predicted_composite(g, rs, sc.human_xy, sc.radius,
                                            sc.height)
        np.testing.assert_array_equal(c, wc)
        np.testing.assert_array_equal(f, wf.view(np.int32))


def test_signed_root_rounding(tmp_path):
    """The signed root's rounding step (device_common.h) against IEEE sqrt:
    start values one ulp off either way, every integer up to 2^22."""
    exe = str(tmp_path / "root_check")
    subprocess.run(["g++", "-O1", "-std=c++20", "-ffp-contract=off",
                    "-I" + os.path.join(HERE, "cpu_device"), "-o", exe,
                    os.path.join(HERE, "cpu_device", "root_check.cpp")],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches 0" in r.stdout

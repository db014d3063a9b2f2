"""Batched composite fields (persistent launches, hipGraph replay,
autotuned launch shapes): outputs must equal one plain call per scene byte
for byte, and the plain call equals the oracle (see test_gpu_parity)."""
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


def static_on_gpu(pc, sc, dev):
    occ = torch.from_numpy(np.ascontiguousarray(sc.occ)).to(dev)
    ssq, _ = pc.build_static_sdf(sc.grid, occ, want_sdf=False)
    return ssq


def scene_dict(pc, sc, dev, static=None):
    return {"grid": sc.grid, "static_ssq": static if static is not None
            else static_on_gpu(pc, sc, dev), "human_xy": sc.human_xy,
            "radius": sc.radius, "height": sc.height}


def plain(pc, d):
    return pc.predicted_composite_sdf(d["grid"], d["static_ssq"],
                                      d["human_xy"], d["radius"],
                                      d["height"])


def ragged_scenes(seed=0):
    # nx*ny odd, divisible by 4 (also with nx odd or 2 mod 4), 2 mod 4,
    # and odd with V divisible by 4: the composite's 1-, 4- and 2-voxel
    # packs, and 4-wide packs whose planar values are gathered
    dims = [(37, 29, 23, 3, 2), (64, 48, 40, 5, 3), (21, 60, 17, 1, 1),
            (100, 36, 30, 7, 4), (8, 8, 8, 2, 0), (130, 70, 33, 4, 2),
            (44, 44, 44, 6, 4), (34, 27, 13, 3, 2), (33, 27, 20, 2, 2)]
    out = []
    for q, (nx, ny, nz, n, K) in enumerate(dims):
        sc = scenegen.small_scene(seed + q, nx, ny, nz, h=0.05, n_boxes=5,
                                  n_humans=max(K, 1), n_slices=n)
        if K == 0:
            sc.human_xy = np.zeros((n, 0, 2))
        out.append(sc)
    return out


def assert_same(outs, refs):
    for q, ((c, f), (rc, rf)) in enumerate(zip(outs, refs)):
        assert torch.equal(c, rc), f"scene {q} int32 differs"
        assert torch.equal(f.view(torch.int32), rf.view(torch.int32)), \
            f"scene {q} fp32 differs"


@pytest.mark.skip(reason="ran the earlier single-launch batch kernel whose "
                  "composite items waited on device flags for their planes; "
                  "it stalled on the GPU twice, the cause was not found, "
                  "and that design was removed (the batch now runs as two "
                  "wait-free persistent launches, tested below)")
def test_batch_matches_plain_and_oracle(pc, dev):
    scs = ragged_scenes()
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    say("batch ragged scenes:", [(s.grid.nx, s.grid.ny, s.grid.nz,
                                  s.n_slices, s.n_humans) for s in scs])
    refs = [plain(pc, d) for d in ds]
    outs = pc.predicted_composite_sdf_batch(ds)
    torch.cuda.synchronize()
    assert_same(outs, refs)
    for sc, (c, f) in zip(scs[:4], outs[:4]):
        rs, _ = oracle.build_static(sc.grid, sc.occ)
        wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy,
                                            sc.radius, sc.height)
        np.testing.assert_array_equal(c.cpu().numpy(), wc)


def test_two_launch_batch_matches_plain_and_oracle(pc, dev):
    scs = ragged_scenes(100)
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    refs = [plain(pc, d) for d in ds]
    torch.cuda.synchronize()
    say("plain calls done; batch of", len(ds), "scenes")
    outs = pc.predicted_composite_sdf_batch(ds)
    torch.cuda.synchronize()
    say("batch done")
    assert_same(outs, refs)
    for sc, (c, f) in zip(scs[:4], outs[:4]):
        rs, _ = oracle.build_static(sc.grid, sc.occ)
        wc, wf = oracle.predicted_composite(sc.grid, rs, sc.human_xy,
                                            sc.radius, sc.height)
        np.testing.assert_array_equal(c.cpu().numpy(), wc)


def test_batch_with_chord_tables_beyond_lds(pc, dev):
    """A scene whose chord table (K x ny pairs) exceeds the planar items'
    LDS takes the path with chords and row passes in global memory, beside
    scenes that keep theirs in LDS."""
    scs = ragged_scenes(200)[:3]
    scs.append(scenegen.small_scene(250, 30, 1000, 6, h=0.05, n_boxes=5,
                                    n_humans=8, n_slices=2))
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    refs = [plain(pc, d) for d in ds]
    torch.cuda.synchronize()
    say("batch with a 30x1000x6 scene of 8 humans")
    outs = pc.predicted_composite_sdf_batch(ds)
    torch.cuda.synchronize()
    assert_same(outs, refs)
    sc = scs[-1]
    rs, _ = oracle.build_static(sc.grid, sc.occ)
    wc, _ = oracle.predicted_composite(sc.grid, rs, sc.human_xy, sc.radius,
                                       sc.height)
    np.testing.assert_array_equal(outs[-1][0].cpu().numpy(), wc)


@pytest.mark.parametrize("G,C,B", [(1, 256, 1), (3, 512, 2), (2, 8192, 4),
                                   (7, 32768, 8), (30, 1024, 32),
                                   (4, 256, 0), (1, 1024, 0), (3, 4096, 0)])
def test_batch_any_tuning_gives_identical_bytes(pc, dev, G, C, B):
    h = pc.Handle()
    h.set_tuning({"batch_slices_per_item": G, "batch_chunk_quads": C,
                  "batch_blocks_per_cu": B})
    scs = ragged_scenes(10)
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    refs = [plain(pc, d) for d in ds]
    say(f"batch tuning G={G} chunk={C} blocks/CU={B}")
    outs = pc.predicted_composite_sdf_batch(ds, handle=h)
    torch.cuda.synchronize()
    assert_same(outs, refs)
    h.close()


def test_batch_graph_replays_and_position_updates(pc, dev):
    scs = ragged_scenes(20)
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    refs = [plain(pc, d) for d in ds]
    g = pc.BatchGraph(ds)
    for r in range(3):
        say("graph replay", r)
        for c, f in g.outputs:       # clobber outputs between replays
            c.fill_(7)
            f.fill_(-1.0)
        x = torch.randn(1 << 20, device=dev)   # unrelated eager work
        (x * 2).sum().item()
        g.launch()
        torch.cuda.synchronize()
        assert_same(g.outputs, refs)
    # new predictions for scene 1 change only scene 1's output
    xy = scs[1].human_xy + np.array([0.3, -0.2])
    g.set_positions(1, xy)
    ds[1]["human_xy"] = xy
    refs[1] = plain(pc, ds[1])
    g.launch()
    torch.cuda.synchronize()
    assert_same(g.outputs, refs)
    g.close()


def test_autotuners_pick_a_shape_with_identical_output(pc, dev):
    h = pc.Handle()
    scs = ragged_scenes(30)
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    refs = [plain(pc, d) for d in ds]
    tun, ms = pc.autotune_batch(ds, reps=1, handle=h)
    say("batch tuning", tun, ms)
    assert ms > 0 and tun["batch_slices_per_item"] > 0
    outs = pc.predicted_composite_sdf_batch(ds, handle=h)
    torch.cuda.synchronize()
    assert_same(outs, refs)
    tun, ms, (c, f) = pc.autotune_composite(ds[3], reps=1, handle=h)
    say("composite tuning", tun, ms)
    assert tun["composite_slices_per_block"] > 0
    assert_same([(c, f)], [refs[3]])
    h.close()


@pytest.mark.slow
def test_batch64_equals_64_plain_calls(pc, dev):
    scs = scenegen.batch64()
    ds = [scene_dict(pc, sc, dev) for sc in scs]
    say("batch64: 64 scenes, voxel-slices =",
        sum(sc.grid.nvox * sc.n_slices for sc in scs))
    outs = pc.predicted_composite_sdf_batch(ds)
    torch.cuda.synchronize()
    for q, d in enumerate(ds):
        rc, rf = plain(pc, d)
        c, f = outs[q]
        assert torch.equal(c, rc), q
        assert torch.equal(f.view(torch.int32), rf.view(torch.int32)), q
        del rc, rf
    g = pc.BatchGraph(ds)
    g.launch()
    torch.cuda.synchronize()
    for q in range(len(ds)):
        assert torch.equal(g.outputs[q][0], outs[q][0]), q
    g.close()

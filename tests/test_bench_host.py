"""Host logic of bench.py that needs no GPU: the traffic records are found
by the run's launch shape and the composite source hash, and a shape or a
source that was not measured gives null."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import bench  # noqa: E402


def _rec(G, order, h, nbytes, V=64, n=5):
    return {"V": V, "n_slices": n, "composite_slices_per_block": G,
            "composite_order": order, "composite_hip_sha256_16": h,
            "bytes_per_launch": nbytes}


def test_traffic_record_by_shape_and_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "traffic_file",
                        lambda w: str(tmp_path / f"{w}.json"))
    h = bench.source_hash(bench.COMPOSITE_SRC)
    bench.store_traffic("w", _rec(1, 0, h, 100.0))
    bench.store_traffic("w", _rec(2, 0, h, 80.0))
    bench.store_traffic("w", _rec(1, 1, h, 60.0))
    bench.store_traffic("w", _rec(2, 0, h, 81.0))  # replaces the shape
    assert bench.load_traffic("w", 64, 5, 2, 0) == 81.0
    assert bench.load_traffic("w", 64, 5, 1, 1) == 60.0
    assert bench.load_traffic("w", 64, 5, 3, 0) is None   # not measured
    assert bench.load_traffic("w", 65, 5, 1, 0) is None   # other grid
    assert sorted(bench.traffic_shapes("w")) == [[1, 0], [1, 1], [2, 0]]
    # a record of another kernel source is dropped on the next store and
    # never reported
    with open(tmp_path / "w.json") as f:
        d = json.load(f)
    d["records"].append(_rec(3, 0, "0" * 16, 50.0))
    with open(tmp_path / "w.json", "w") as f:
        json.dump(d, f)
    assert bench.load_traffic("w", 64, 5, 3, 0) is None
    bench.store_traffic("w", _rec(4, 0, h, 40.0))
    assert [3, 0] not in bench.traffic_shapes("w")
    assert len(bench.traffic_records("w")) == 4

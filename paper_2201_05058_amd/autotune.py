"""JSON cache of the autotuner's launch shapes.

The tuning itself runs in the library (pcsdf_autotune_batch and
pcsdf_autotune_composite time candidate shapes with HIP events on the
caller's real inputs).  This module only remembers the winner per
(device architecture, workload signature) in a JSON file and applies it to
a handle, so a workload is timed once per machine.  A missing or corrupt
cache file is ignored (the library defaults are used and the file is
rewritten).
"""
from __future__ import annotations

import json
import os

DEFAULT_PATH = os.environ.get(
    "PCSDF_TUNING_CACHE",
    os.path.join(os.path.expanduser("~"), ".cache", "pcsdf", "tuning.json"))


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, d: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def composite_signature(grid, n_slices: int, n_humans: int) -> str:
    return f"composite:{grid.nx}x{grid.ny}x{grid.nz}:n{n_slices}:k{n_humans}"


def batch_signature(scenes) -> str:
    vox = sum(s["grid"].nx * s["grid"].ny * s["grid"].nz *
              len(s["human_xy"]) for s in scenes)
    return f"batch:{len(scenes)}:{vox}"


def tuned(handle, signature: str, run_tuner, path: str = DEFAULT_PATH):
    """Applies the cached shape for `signature` to `handle`, or calls
    run_tuner() (which tunes the handle and returns (tuning dict, ms)) and
    caches its result.  Returns (tuning dict, ms or None, from_cache)."""
    key = f"{_arch()}:{signature}"
    cache = _load(path)
    hit = cache.get(key)
    if isinstance(hit, dict) and "tuning" in hit:
        try:
            handle.set_tuning(hit["tuning"])
            return hit["tuning"], hit.get("ms"), True
        except Exception:
            pass
    tun, ms = run_tuner()
    cache[key] = {"tuning": tun, "ms": ms}
    _store(path, cache)
    return tun, ms, False

#!/usr/bin/env python3
"""Throughput of the predicted composite distance field on one MI355X.

One step = the whole hot path over one batch of synthetic input: the
per-slice composite fields of a 512x512x256 grid at 0.01 m (200 static
boxes, 8 humans on piecewise-linear paths, 50 slices at dt = 0.05 s; the
static field is built once beforehand, as the paper's environment field
is) and 100k exact sphere queries per slice (5M) on those fields.
`--workload room256` times the 256x256x128 grid (40 boxes, 3
constant-velocity humans, 20 slices at 0.1 s, 10k spheres) instead; it is
also measured as a section of the default run.

Prints one JSON line.  `value` is voxel-slices/s of whole steps with the
inputs resident in HBM.  `roofline` covers the dominant kernel (the
streaming composite), timed with HIP events on its own launch stream.
`cpu_baseline` times the CPU oracle on a sample of the same workload
(rank 0, N=1), on one core and on all the cores it may use.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("composite-EDT voxel-slices/s (% HBM peak); "
          "sphere queries/s surrogate vs exact")
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "room512": "512x512x256 grid at 0.01 m, 200 seeded boxes, 8 cylinder "
               "humans on piecewise-linear paths, 50 slices at dt=0.05 s, "
               "100k exact sphere queries per slice (5M)",
    "room256": "256x256x128 grid at 0.02 m, 40 seeded boxes, 3 "
               "constant-velocity cylinder humans, 20 slices at dt=0.1 s, "
               "10k exact sphere queries",
}


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles",
                        f"composite_{workload}_traffic.json")

COMPOSITE_SRC = os.path.join(ROOT, "paper_2201_05058_amd", "csrc",
                             "composite.hip")


def source_hash(path: str) -> str:
    """Hash of the composite kernels' own source text (k_static16 and the
    k_composite template, the shared epilogue in composite_device.h and the
    helpers of device_common.h), so host-side edits of composite.hip keep a
    measurement valid."""
    with open(path) as f:
        src = f.read()
    a = src.find("// The 16-bit copy of the static field: S16[v]")
    b = src.find("template <int VEC, bool kGather>", a)
    text = src[a:b] if a >= 0 and b > a else src
    for dep in ("composite_device.h", "device_common.h"):
        with open(os.path.join(os.path.dirname(path), dep)) as f:
            text += f.read()
    return hashlib.sha256(text.encode()).hexdigest()[:16]


def composite_outputs(torch, n, shape_zyx, dev):
    """The composite calls' default output layout (the package's
    composite_outputs: both fields in one allocation, 4 KiB apart)."""
    import paper_2201_05058_amd as pc
    return pc.composite_outputs(n, shape_zyx, dev)


def traffic_from(prof_dir: str, V: int, n: int) -> dict:
    """HBM bytes per composite call from two rocprofv3 --pmc runs
    (FETCH_SIZE and WRITE_SIZE, KiB per dispatch) of this benchmark and of
    a 1 GiB device copy (--calibrate-copy-mib 1024), each counter scaled
    by copy bytes / what it reads for the copy: the k_composite launch
    and, when the call makes one, the k_static16 launch of its 16-bit
    static copy."""
    import csv
    import statistics

    def load(sub):
        # per kernel: {grid size: [counter values]}
        d = {}
        path = None
        for root, _, files in os.walk(os.path.join(prof_dir, sub)):
            for fn in files:
                if fn.endswith("counter_collection.csv"):
                    path = os.path.join(root, fn)
        for r in csv.DictReader(open(path)):
            d.setdefault(r["Kernel_Name"], {}).setdefault(
                int(r["Grid_Size"]), []).append(float(r["Counter_Value"]))
        return d

    def step_launches(d, kernel="k_composite"):
        # the timed step's launch shape: the one dispatched most often
        by_grid = d.get(kernel)
        if not by_grid:
            return None, [0.0]
        g = max(by_grid, key=lambda k: len(by_grid[k]))
        return g, by_grid[g]
    f, w = load("prof_fetch"), load("prof_write")
    cf, cw = load("prof_cfetch"), load("prof_cwrite")
    ck = [k for k in cf if "copyBuffer" in k][0]
    copy = 1024 * 2 ** 20
    fs = copy / (statistics.mean(sum(cf[ck].values(), [])) * 1024)
    ws = copy / (statistics.mean(sum(cw[ck].values(), [])) * 1024)
    grid, fv = step_launches(f)
    _, wv = step_launches(w)
    fb = statistics.mean(fv) * 1024 * fs
    wb = statistics.mean(wv) * 1024 * ws
    _, f16 = step_launches(f, "k_static16")
    _, w16 = step_launches(w, "k_static16")
    fb16 = statistics.mean(f16) * 1024 * fs
    wb16 = statistics.mean(w16) * 1024 * ws
    return {"kernel": "k_composite", "V": V, "n_slices": n,
            "grid_size": grid, "launches": len(fv),
            "fetch_bytes": fb, "write_bytes": wb,
            "static16_fetch_bytes": fb16, "static16_write_bytes": wb16,
            "bytes_per_launch": fb + wb + fb16 + wb16, "fetch_scale": fs,
            "write_scale": ws,
            "composite_hip_sha256_16": source_hash(COMPOSITE_SRC)}


def traffic_records(workload: str) -> list:
    """The traffic records of a workload: one per launch shape measured
    (a file holding a single record is read as a list of one)."""
    try:
        with open(traffic_file(workload)) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return []
    if isinstance(t, dict) and isinstance(t.get("records"), list):
        return [r for r in t["records"] if isinstance(r, dict)]
    return [t] if isinstance(t, dict) else []


def store_traffic(workload: str, rec: dict) -> None:
    """Adds a record, replacing one of the same shape and dropping those
    of other kernel sources."""
    key = (rec.get("composite_slices_per_block"), rec.get("composite_order"))
    recs = [r for r in traffic_records(workload)
            if r.get("composite_hip_sha256_16") ==
            rec["composite_hip_sha256_16"] and
            (r.get("composite_slices_per_block"),
             r.get("composite_order")) != key]
    recs.append(rec)
    recs.sort(key=lambda r: (r.get("composite_order") or 0,
                             r.get("composite_slices_per_block") or 0))
    with open(traffic_file(workload), "w") as fh:
        json.dump({"records": recs}, fh, indent=1)


def load_traffic(workload: str, V: int, n: int, G: int, order: int):
    """Measured HBM bytes per composite call (rocprofv3 PMC FETCH_SIZE +
    WRITE_SIZE, scaled by a copy-kernel calibration) in the launch shape
    of this run (G slices per block row, block order), or None when that
    shape was not measured or the counters were taken on a different
    version of the kernel source."""
    h = source_hash(COMPOSITE_SRC)
    for t in traffic_records(workload):
        if (t.get("composite_hip_sha256_16") == h and t.get("V") == V and
                t.get("n_slices") == n and
                t.get("composite_slices_per_block") == G and
                t.get("composite_order") == order):
            return t.get("bytes_per_launch")
    return None


def traffic_shapes(workload: str) -> list:
    """[G, order] of every measured shape whose source hash matches."""
    h = source_hash(COMPOSITE_SRC)
    return [[t.get("composite_slices_per_block"), t.get("composite_order")]
            for t in traffic_records(workload)
            if t.get("composite_hip_sha256_16") == h]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(sc, single_slices: int, omp_slices: int, runs: int = 3):
    """The oracle on a bounded sample of the workload: the first
    `single_slices` slices on one core (one run), and the first
    `omp_slices` slices with the same C built with OpenMP on every core it
    may use (median of `runs`).  The static field (not part of a step) is
    built beforehand by the OpenMP build."""
    import statistics
    import oracle
    rs, _ = oracle.build_static(sc.grid, sc.occ, omp=True)
    V = sc.grid.nvox

    def once(n, omp):
        t0 = time.perf_counter()
        oracle.predicted_composite(sc.grid, rs, sc.human_xy[:n], sc.radius,
                                   sc.height, omp=omp)
        return time.perf_counter() - t0
    n1 = min(single_slices, sc.n_slices)
    t1 = once(n1, False)
    nm = min(omp_slices, sc.n_slices)
    tm = statistics.median(once(nm, True) for _ in range(runs))
    threads = oracle.threads(omp=True)
    return {"value": V * nm / tm, "unit": "voxel-slices/s",
            "cores": threads, "kind": "oracle",
            "sample": f"slices 0-{nm - 1} of {sc.n_slices} of the same "
                      f"workload, OpenMP build of the C oracle on {threads} "
                      f"threads, median of {runs} runs of {tm:.2f} s",
            "cpu_model": cpu_model(),
            "cores_available": len(os.sched_getaffinity(0)),
            "single_thread": {
                "value": V * n1 / t1, "unit": "voxel-slices/s", "cores": 1,
                "sample": f"slice{'s 0-' if n1 > 1 else ' '}"
                          f"{n1 - 1 if n1 > 1 else 0} of {sc.n_slices}, "
                          f"plain single-threaded build, one run of "
                          f"{t1:.2f} s"}}


def batch_section(pc, autotune, scenegen, torch, dev, reps: int = 5):
    """64 uneven scenes (5-30 slices, 1-4 humans, grids 64..256 x 64..256 x
    64..128 at 0.02-0.05 m): one captured hipGraph replay of the batch
    against 64 plain calls on one stream, same outputs, by wall time and by
    GPU time (the plain calls' wall time includes the host's per-call
    work).  Static fields are built before timing; their GPU time is
    reported beside it (the variant that includes them)."""
    from paper_2201_05058_amd import _native
    scs = scenegen.batch64()
    h = pc.Handle()
    scenes = []
    occ0 = torch.from_numpy(scs[0].occ).to(dev)  # warm the static kernels
    pc.build_static_sdf(scs[0].grid, occ0, want_sdf=False, handle=h)
    torch.cuda.synchronize()
    del occ0
    h.profile(True)
    h.profile_reset()
    for sc in scs:
        occ = torch.from_numpy(sc.occ).to(dev)
        ssq, _ = pc.build_static_sdf(sc.grid, occ, want_sdf=False, handle=h)
        del occ
        oc, of = composite_outputs(torch, sc.n_slices, sc.grid.shape_zyx,
                                   dev)
        scenes.append({"grid": sc.grid, "static_ssq": ssq,
                       "human_xy": sc.human_xy, "radius": sc.radius,
                       "height": sc.height, "out_ssq": oc, "out_sdf": of})
    torch.cuda.synchronize()
    static_gpu = h.profile_read(_native.KERNEL_STATIC)[0]
    h.profile(False)
    vs = sum(sc.grid.nvox * sc.n_slices for sc in scs)
    tuning, _, _ = autotune.tuned(
        h, autotune.batch_signature(scenes),
        lambda: pc.autotune_batch(scenes, reps=2, handle=h))
    graph = pc.BatchGraph(scenes, handle=h)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    def plain_all():
        for d in scenes:
            pc.predicted_composite_sdf(d["grid"], d["static_ssq"],
                                       d["human_xy"], d["radius"],
                                       d["height"], out_ssq=d["out_ssq"],
                                       out_sdf=d["out_sdf"], handle=h)

    g_ms = timed(graph.launch)
    p_ms = timed(plain_all)
    # GPU time alone (HIP events on the stream around each library call):
    # the plain calls' wall time also holds the host's per-call work
    h.profile(True)
    h.profile_reset()
    timed(graph.launch)
    g_gpu = h.profile_read(_native.KERNEL_BATCH)[0] / (reps + 1)
    h.profile_reset()
    timed(plain_all)
    p_gpu = sum(h.profile_read(k)[0] for k in (_native.KERNEL_PLANES,
                                               _native.KERNEL_COMPOSITE))
    p_gpu /= reps + 1
    h.profile(False)
    graph.close()
    h.close()
    return {"scenes": len(scs), "voxel_slices": vs,
            "graph_ms": g_ms, "plain_64_calls_ms": p_ms,
            "graph_gpu_ms": g_gpu, "plain_64_calls_gpu_ms": p_gpu,
            "static_builds_64_gpu_ms": static_gpu,
            "graph_plus_static_builds_gpu_ms": g_gpu + static_gpu,
            "speedup_vs_plain_gpu": p_gpu / g_gpu,
            "graph_voxel_slices_per_s": vs / (g_ms / 1e3),
            "plain_voxel_slices_per_s": vs / (p_ms / 1e3),
            "speedup_vs_plain": p_ms / g_ms,
            "graph_gbs_8B_basis": 8.0 * vs / (g_ms / 1e3) / 1e9,
            "tuning": tuning}


def measure_workload(pc, autotune, torch, dev, sc, name: str, steps: int,
                     warmup: int, sections=None):
    """Whole steps of one workload (composite of every slice, then the exact
    sphere queries on the fields): wall time per step over `steps` timed
    steps, the composite kernel's own time during them (HIP events of its
    dispatch on the launch stream), then the planes and the queries timed
    over as many steps right after.  The static build (once per scene) is
    timed apart.  `sections(h, occ, ssq_s, out_ssq, out_sdf)` may add
    measurements on the same buffers; its dict is merged into the result."""
    from paper_2201_05058_amd import _native
    g = sc.grid
    V, n, K = g.nvox, sc.n_slices, sc.n_humans
    q = sc.queries
    Q = len(q.radius)
    h = pc.Handle()
    occ = torch.from_numpy(sc.occ).to(dev)
    centre = torch.from_numpy(q.centre).to(dev)
    radius = torch.from_numpy(q.radius).to(dev)
    slices = torch.from_numpy(q.slice).to(dev)
    out_ssq, out_sdf = composite_outputs(torch, n, g.shape_zyx, dev)

    # static field, built once per scene (not part of a step); timed warm
    # over three builds with both outputs
    h.profile(True)
    ssq_s, sdf_s = pc.build_static_sdf(g, occ, handle=h)
    torch.cuda.synchronize()
    h.profile_reset()
    for _ in range(3):
        pc.build_static_sdf(g, occ, ssq=ssq_s, sdf=sdf_s, handle=h)
    torch.cuda.synchronize()
    st_ms, st_n = h.profile_read(_native.KERNEL_STATIC)
    static_ms = st_ms / max(st_n, 1)
    del sdf_s

    # launch shape of the composite, tuned on this workload (cached)
    scene = {"grid": g, "static_ssq": ssq_s, "human_xy": sc.human_xy,
             "radius": sc.radius, "height": sc.height, "out_ssq": out_ssq,
             "out_sdf": out_sdf}
    tuning, _, _ = autotune.tuned(
        h, autotune.composite_signature(g, n, K),
        lambda: pc.autotune_composite(scene, reps=3 if V * n < 1e9 else 2,
                                      handle=h)[:2])

    def step():
        pc.predicted_composite_sdf(g, ssq_s, sc.human_xy, sc.radius,
                                   sc.height, out_ssq=out_ssq,
                                   out_sdf=out_sdf, handle=h)
        return pc.query_spheres(g, out_sdf, centre, radius, slices,
                                handle=h)

    # The timed steps time the composite kernel alone (a timed kernel
    # costs the stream a few microseconds before it); the planes and
    # queries are timed over as many steps right after.
    h.profile(True, only=[_native.KERNEL_COMPOSITE])
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    h.profile_reset()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    comp_ms, comp_n = h.profile_read(_native.KERNEL_COMPOSITE)

    h.profile(True, only=[_native.KERNEL_PLANES, _native.KERNEL_QUERY])
    h.profile_reset()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    pl_ms, pl_n = h.profile_read(_native.KERNEL_PLANES)
    qy_ms, qy_n = h.profile_read(_native.KERNEL_QUERY)
    h.profile(True)
    comp_avg_s = comp_ms / comp_n / 1e3
    # compulsory bytes of one composite call: read the static field once
    # (4 B/voxel) and write both outputs (8 B/voxel-slice).  The call's
    # time is that of its kernels: k_composite and, when it makes the
    # 16-bit static copy, k_static16 before it.
    alg_bytes = (8.0 + 4.0 / n) * V * n
    achieved = alg_bytes / comp_avg_s / 1e9
    # the library's rule for the copy (pcsdf_tuning.composite_static16)
    G = min(tuning.get("composite_slices_per_block") or 2, n)
    order = int(tuning.get("composite_order") or 0)
    c16 = tuning.get("composite_static16", 0)
    copy16 = c16 == 2 or (c16 == 0 and V >= 1 << 25 and -(-n // G) >= 4)
    qy_avg = qy_ms / max(qy_n, 1)
    res = {
        "value": V * n / (ms_per_step / 1e3),
        "ms_per_step": ms_per_step,
        "config": {"workload": WORKLOADS[name],
                   "grid": [g.nx, g.ny, g.nz], "voxel_m": g.h,
                   "n_slices": n, "n_humans": K, "n_queries": Q,
                   "seed": sc.seed},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            # counters of this run's launch shape (the static re-reads
            # scale with the slice groups), null for a shape not measured
            "traffic": load_traffic(name, V, n, G, order),
            "traffic_shapes_measured": traffic_shapes(name),
            "composite_slices_per_block": G,
            "composite_order": order,
            "kernel": ("k_static16 + k_composite" if copy16
                       else "k_composite"),
            "kernel_ms": comp_avg_s * 1e3,
            "kernel_launches_timed": comp_n,
            "bytes_per_voxel_slice": 8.0 + 4.0 / n,
            "frac_12B_basis": 12.0 * V * n / comp_avg_s / 1e9 / HBM_PEAK_GBS,
        },
        "kernels_ms": {"composite": comp_avg_s * 1e3,
                       "planes": pl_ms / max(pl_n, 1),
                       "query": qy_avg,
                       "static_build_once": static_ms},
        "static_build_gbs_9B_basis": 9.0 * V / (static_ms * 1e-3) / 1e9,
        "queries_per_s_exact_kernel": Q / (qy_avg / 1e3)
        if qy_ms > 0 else None,
        "tuning": tuning,
    }
    if sections is not None:
        res.update(sections(h, occ, ssq_s, out_ssq, out_sdf))
    del out_ssq, out_sdf
    torch.cuda.empty_cache()
    # exact queries answered without fields (planes + static field only)
    pc.query_spheres_direct(g, ssq_s, sc.human_xy, sc.radius, sc.height,
                            centre, radius, slices, handle=h)
    torch.cuda.synchronize()
    h.profile(True, only=[_native.KERNEL_PLANES, _native.KERNEL_QUERY])
    h.profile_reset()
    reps = 3
    for _ in range(reps):
        pc.query_spheres_direct(g, ssq_s, sc.human_xy, sc.radius, sc.height,
                                centre, radius, slices, handle=h)
    torch.cuda.synchronize()
    res["direct_query_ms_incl_planes"] = (
        h.profile_read(_native.KERNEL_QUERY)[0] +
        h.profile_read(_native.KERNEL_PLANES)[0]) / reps
    h.close()
    del occ, ssq_s
    torch.cuda.empty_cache()
    return res


def next_rows_section(pc, torch, sc, occ, ssq_s, out_ssq, out_sdf, h,
                      reps: int = 5):
    """The adjacent variants on the same workload, by GPU time: the
    composite with radii growing over the horizon (r0 + 0.05 m/s * t), the
    map collapsed to the floor plane and its 2-D signed EDT, and GPMP2
    obstacle factors (hinge errors, Jacobians, per-state costs) of 64
    spheres at 100 support states spread over the 20 slices."""
    import numpy as np
    from paper_2201_05058_amd import _native
    g = sc.grid
    n = sc.n_slices
    dev = ssq_s.device
    radii = sc.radius + 0.05 * sc.dt * np.arange(n)

    def grow():
        pc.predicted_composite_sdf_growing(g, ssq_s, sc.human_xy, radii,
                                           sc.height, out_ssq=out_ssq,
                                           out_sdf=out_sdf, handle=h)
    grow()
    torch.cuda.synchronize()
    h.profile_reset()
    for _ in range(reps):
        grow()
    torch.cuda.synchronize()
    grow_ms = (h.profile_read(_native.KERNEL_COMPOSITE)[0] +
               h.profile_read(_native.KERNEL_PLANES)[0]) / reps

    def stream_ms(fn):
        fn()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) / reps
    floor_ms = stream_ms(lambda: pc.build_floor_sdf(g, occ, handle=h))

    S, J = 100, 64
    rng = np.random.Generator(np.random.PCG64(9))
    lo = np.array(g.origin) + 0.1
    span = np.array(g.extent) - 0.2
    centre = torch.from_numpy((rng.random((S, J, 3)) * span + lo)
                              .astype(np.float32)).to(dev)
    radius = torch.from_numpy(rng.uniform(0.05, 0.15, J)
                              .astype(np.float32)).to(dev)
    st_slice = torch.from_numpy((np.arange(S) * n // S)
                                .astype(np.int32)).to(dev)
    pc.obstacle_factors(g, out_sdf, centre, radius, st_slice, 0.2, 0.1,
                        handle=h)
    torch.cuda.synchronize()
    h.profile_reset()
    for _ in range(reps):
        pc.obstacle_factors(g, out_sdf, centre, radius, st_slice, 0.2, 0.1,
                            handle=h)
    torch.cuda.synchronize()
    fac_ms = h.profile_read(_native.KERNEL_FACTORS)[0] / reps
    return {"growing_radius_composite_ms": grow_ms,
            "growing_radius_voxel_slices_per_s": g.nvox * n / (grow_ms / 1e3),
            "floor_edt_ms": floor_ms, "floor_grid": [g.nx, g.ny],
            "obstacle_factors_ms": fac_ms,
            "obstacle_factors_sphere_states": S * J,
            "sphere_states_per_s": S * J / (fac_ms / 1e3)}


def recompute_section(pc, torch, sc, occ, ssq_s, out_ssq, out_sdf, h,
                      reps: int = 3):
    """The paper's composite benchmark (mapping section, Fig. 6) on this
    workload: the composite call against recomputing every slice's field
    from scratch (exact signed EDT of the environment and the humans' voxels
    with this library's three-pass EDT), without and with copying the n
    fp32 fields to pinned host memory afterwards."""
    g = sc.grid
    host = torch.empty(tuple(out_sdf.shape), dtype=torch.float32,
                       pin_memory=True)

    def comp():
        pc.predicted_composite_sdf(g, ssq_s, sc.human_xy, sc.radius,
                                   sc.height, out_ssq=out_ssq,
                                   out_sdf=out_sdf, handle=h)

    def reco():
        pc.recompute_sdf(g, occ, sc.human_xy, sc.radius, sc.height,
                         out_ssq=out_ssq, out_sdf=out_sdf, handle=h)

    def copied(fn):
        def run():
            fn()
            host.copy_(out_sdf, non_blocking=True)
        return run

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    c_ms, r_ms = timed(comp), timed(reco)
    cc_ms, rc_ms = timed(copied(comp)), timed(copied(reco))
    del host
    return {"slices": sc.n_slices, "composite_ms": c_ms,
            "recompute_ms": r_ms, "speedup_excl_copy": r_ms / c_ms,
            "composite_with_copy_ms": cc_ms,
            "recompute_with_copy_ms": rc_ms,
            "speedup_incl_copy": rc_ms / cc_ms,
            "copy_bytes": out_sdf.numel() * 4,
            "copy_gbs": out_sdf.numel() * 4 / ((cc_ms - c_ms) / 1e3) / 1e9
            if cc_ms > c_ms else None,
            "paper_context": "9.1-13.6x excluding and 1.7-2.1x including "
                             "the device-to-host copy, against PBA on an "
                             "RTX 2060 (grid sizes not recoverable)"}


def template_section(pc, torch, sc, ssq_s, out_ssq, out_sdf, h,
                     reps: int = 5):
    """The mapping section's own placement (each human's cylinder field
    computed once and shifted by whole voxels per slice) against the exact
    per-slice composite on this workload: time of each call and how far the
    shifted templates are from the exact fields."""
    g = sc.grid

    def exact():
        pc.predicted_composite_sdf(g, ssq_s, sc.human_xy, sc.radius,
                                   sc.height, out_ssq=out_ssq,
                                   out_sdf=out_sdf, handle=h)

    def tmpl():
        pc.template_composite_sdf(g, ssq_s, sc.human_xy, sc.radius,
                                  sc.height, out_ssq=out_ssq,
                                  out_sdf=out_sdf, handle=h)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    e_ms, t_ms = timed(exact), timed(tmpl)
    h.profile_reset()
    tmpl()
    torch.cuda.synchronize()
    from paper_2201_05058_amd import _native
    k_ms, k_n = h.profile_read(_native.KERNEL_TEMPLATE)
    k_ms /= max(k_n, 1)
    exact()
    ref = out_sdf.clone()
    tmpl()
    torch.cuda.synchronize()
    fin = torch.isfinite(ref) & torch.isfinite(out_sdf)
    d = (out_sdf - ref).abs()[fin]
    differ = float((out_sdf != ref).float().mean())
    V, n = g.nvox, sc.n_slices
    res = {"exact_call_ms": e_ms, "template_call_ms": t_ms,
           "template_kernel_ms": k_ms,
           "template_kernel_gbs_8B_basis":
               (8.0 + 4.0 / n) * V * n / (k_ms / 1e3) / 1e9,
           "voxels_differing": differ,
           "max_abs_diff_m": float(d.max()), "mean_abs_diff_m":
               float(d.mean())}
    del ref
    return res


def surrogate_section(pc, torch, dev, room: str, weights: str):
    """Sphere queries by the trained per-human surrogate (with exact
    fallback) against the exact path on the room's evaluation workload
    (room256: 1M spheres, three fresh constant-velocity humans; room512:
    its 5M spheres and eight piecewise-linear humans): error in metres on
    the queries it answers, the fallback fraction, and GPU time of both
    paths."""
    from paper_2201_05058_amd import train
    if not os.path.exists(weights):
        return {"weights": None, "note": "no trained weights file"}
    net, meta = train.load(weights)
    sc = train.evaluation_scene(room)
    res = train.evaluate(net, sc, dev)
    res["queries_per_s_surrogate"] = res["queries"] / (
        res["surrogate_path_ms"] / 1e3)
    res["queries_per_s_exact_direct"] = res["queries"] / (
        res["exact_direct_ms"] / 1e3)
    res["weights"] = os.path.relpath(weights, ROOT)
    res["trained_on"] = meta
    net.close()
    del sc
    torch.cuda.empty_cache()
    return res


def hbm_ceilings(mib: int = 1024, reps: int = 20):
    """Plain torch kernels on buffers of `mib` MiB: fill (write only), sum
    (read only) and copy, best of `reps` timed with CUDA events: the
    bandwidths a streaming kernel can reach on this GPU."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    out = {"buffer_bytes": n * 4}
    cases = {"write_fill": (lambda: a.fill_(1.0), n * 4),
             "read_sum": (lambda: a.sum(), n * 4),
             "copy": (lambda: b.copy_(a), 2 * n * 4)}
    for name, (fn, nbytes) in cases.items():
        fn()
        torch.cuda.synchronize()
        best = None
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ms = e0.elapsed_time(e1)
            best = ms if best is None else min(best, ms)
        out[name + "_gbs"] = nbytes / (best / 1e3) / 1e9
    print(json.dumps(out))


def mlp_rows(n: int, weights: str, reps: int = 10):
    """The fused surrogate network (value and input gradient) on n seeded
    rows of its 16 features, kernel time by the library's HIP events."""
    import numpy as np
    import torch
    from paper_2201_05058_amd import _native, train
    torch.cuda.set_device(0)
    net, _ = train.load(weights)
    rng = np.random.default_rng(0)
    x = torch.from_numpy(
        (rng.normal(size=(n, net.n_in)) * 3).astype(np.float32)).cuda()
    net.forward(x)
    torch.cuda.synchronize()
    best = None
    for _ in range(3):
        net.h.profile(True, only=[_native.KERNEL_MLP])
        net.h.profile_reset()
        for _ in range(reps):
            net.forward(x)
        torch.cuda.synchronize()
        ms = net.h.profile_read(_native.KERNEL_MLP)[0] / reps
        best = ms if best is None else min(best, ms)
    net.h.profile(False)
    flop = 205056 * n
    print(json.dumps({"mlp_rows": n, "kernel": "k_mlp_infer", "ms": best,
                      "tflops": flop / (best / 1e3) / 1e12,
                      "frac_bf16_dense": flop / (best / 1e3) / 2.5e15}))
    net.close()


def static_builds(workloads, reps: int):
    """The static build (pcsdf_build_static_sdf) of each workload's map,
    `reps` builds per round, three rounds: the best round's mean build
    time by the library's HIP events (kernel-trace and counter runs use
    this mode)."""
    import torch

    import paper_2201_05058_amd as pc
    import scenegen
    from paper_2201_05058_amd import _native
    torch.cuda.set_device(0)
    out = {}
    for name in workloads:
        sc = (scenegen.room256() if name == "room256"
              else scenegen.room512(with_queries=False))
        occ = torch.from_numpy(sc.occ).cuda()
        h = pc.Handle()
        pc.build_static_sdf(sc.grid, occ, handle=h)
        torch.cuda.synchronize()
        best = None
        for _ in range(3):
            h.profile(True, only=[_native.KERNEL_STATIC])
            h.profile_reset()
            for _ in range(reps):
                pc.build_static_sdf(sc.grid, occ, handle=h)
            torch.cuda.synchronize()
            ms = h.profile_read(_native.KERNEL_STATIC)[0] / reps
            best = ms if best is None else min(best, ms)
        h.profile(False)
        h.close()
        out[name + "_static_build_ms"] = best
        del occ
        torch.cuda.empty_cache()
    print(json.dumps(out))


def calibrate_copy(mib: int, reps: int):
    """A plain device copy of known size, for scaling PMC byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration_copy_bytes": n * 4, "reps": reps}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=sorted(WORKLOADS),
                    default="room512")
    ap.add_argument("--cpu-slices", type=int, default=1,
                    help="slices of the single-threaded oracle sample")
    ap.add_argument("--cpu-omp-slices", type=int, default=4,
                    help="slices of the all-core oracle sample")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0)
    ap.add_argument("--hbm-ceilings", action="store_true",
                    help="measure fill, sum and copy bandwidths and exit")
    ap.add_argument("--mlp-rows", type=int, default=0,
                    help="time the fused surrogate network on this many "
                         "rows and exit")
    ap.add_argument("--static-builds", type=int, default=0,
                    help="time this many static builds per round of the "
                         "256x256x128 and 512x512x256 maps and exit")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-scene batch measurement")
    ap.add_argument("--no-room256", action="store_true",
                    help="skip the 256x256x128 x 20-slice section")
    ap.add_argument("--no-recompute", action="store_true",
                    help="skip the composite vs full recompute measurement")
    ap.add_argument("--no-surrogate", action="store_true",
                    help="skip the surrogate query measurement")
    ap.add_argument("--weights-dir", default=os.path.join(
        ROOT, "paper_2201_05058_amd", "weights"))
    ap.add_argument("--traffic-shape", default="2,0",
                    help="slices per block row and block order of the "
                    "launches whose counters --traffic-from reads (the "
                    "tuning the counted runs were given)")
    ap.add_argument("--traffic-from", default="",
                    help="write the composite's measured HBM traffic from "
                         "rocprofv3 PMC output under this directory")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not "
              f"supported (slices shard across GPUs by design, but the "
              f"library has no multi-GPU path).", file=sys.stderr)
        sys.exit(2)
    if args.hbm_ceilings:
        hbm_ceilings()
        return
    if args.mlp_rows:
        mlp_rows(args.mlp_rows, os.path.join(args.weights_dir,
                                             "surrogate_room256.npz"))
        return
    if args.static_builds:
        static_builds(["room256", "room512"], args.static_builds)
        return
    if args.calibrate_copy_mib:
        calibrate_copy(args.calibrate_copy_mib, max(1, args.steps))
        return
    if args.traffic_from:
        V, n = {"room512": (512 * 512 * 256, 50),
                "room256": (256 * 256 * 128, 20)}[args.workload]
        t = traffic_from(args.traffic_from, V, n)
        G, order = (int(x) for x in args.traffic_shape.split(","))
        t["composite_slices_per_block"] = G
        t["composite_order"] = order
        store_traffic(args.workload, t)
        print(json.dumps(t))
        return

    import torch

    import paper_2201_05058_amd as pc
    import scenegen
    from paper_2201_05058_amd import autotune

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    make = {"room512": scenegen.room512, "room256": scenegen.room256}
    sc = make[args.workload]()
    head = measure_workload(pc, autotune, torch, dev, sc, args.workload,
                            args.steps, args.warmup)

    line = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "voxel-slices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": head.pop("config"),
        "roofline": head.pop("roofline"),
    }
    line.update(head)
    if args.workload != "room256" and not args.no_room256:
        sc2 = scenegen.room256()

        def sections(h, occ, ssq_s, out_ssq, out_sdf):
            if args.no_recompute:
                return {}
            return {"fig6_recompute": recompute_section(
                        pc, torch, sc2, occ, ssq_s, out_ssq, out_sdf, h),
                    "template_composite": template_section(
                        pc, torch, sc2, ssq_s, out_ssq, out_sdf, h),
                    "next_rows": next_rows_section(
                        pc, torch, sc2, occ, ssq_s, out_ssq, out_sdf, h)}
        line["room256"] = measure_workload(
            pc, autotune, torch, dev, sc2, "room256", args.steps,
            args.warmup, sections)
    if not args.no_surrogate:
        for room in ("room256", "room512"):
            line[f"surrogate_{room}"] = surrogate_section(
                pc, torch, dev, room,
                os.path.join(args.weights_dir, f"surrogate_{room}.npz"))
    if not args.no_batch:
        line["batch64"] = batch_section(pc, autotune, scenegen, torch,
                                        dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(sc, args.cpu_slices,
                                            args.cpu_omp_slices)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Trainer of the per-human sphere-query surrogate.

The network answers one (query, human) row: the exact field of a single
human at the query, as a residual over the distance d to the continuous
cylinder (pcsdf_query_spheres_surrogate, oracle/surrogate.py).  The row's
features are relative to the human and in voxel units, so one network
serves every room with the same voxel size, cylinder radius and top layer
(room256: 0.02 m voxels; room512: 0.01 m), any number of humans and any
path model.

Each step of the data pipeline and of the optimisation runs in the
library's kernels.  A pool of P single-human configurations is kept, each
a whole disk inside an empty room of the target grid (one human per slice
of a P-slice call); every step replaces one configuration, labels a batch
of sphere centres around the pool's humans with the exact distance at the
centre (pcsdf_query_spheres_direct on an all-free environment, zero
radius), turns them into rows and residual targets
(pcsdf_surrogate_human_features) and takes one Adam step on the squared
error in voxels (pcsdf_mlp_train_step).  This module draws the random
inputs (positions on the host, offsets with a seeded torch generator on
the device) and sequences the calls.

Checkpoints (save_checkpoint / resume) hold the optimiser's whole state
(fp32 masters, Adam moments, step), the pool, both random generators and
the schedule, so a resumed run continues exactly as the uninterrupted one.

Usage:  python -m paper_2201_05058_amd.train --room room512 --out w.npz
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

import scenegen

from . import build_static_sdf, default_handle, query_spheres_direct
from .surrogate import (NIN, Mlp, init_params, query_spheres_surrogate,
                        surrogate_human_features)

# Name of the row transform (pcsdf_surrogate_human_features): weights
# trained on another transform are refused by load().
FEATURES = "per-human-residual-v1"
ROOMS = {"room256": scenegen.room256, "room512": scenegen.room512}


def room_grid(name: str):
    if name == "room512":
        return scenegen.room512(with_queries=False)
    return scenegen.room256(n_queries=0)


class Trainer:
    """State of one training run (everything a checkpoint holds)."""

    def __init__(self, grid, dev, radius=scenegen.HUMAN_RADIUS,
                 height=scenegen.HUMAN_HEIGHT, pool=32, batch=32768,
                 steps=10000, lr=1e-3, lr_min=1e-5, seed=0, near=0.6,
                 reach=1.5):
        import torch
        self.grid, self.dev = grid, dev
        self.radius, self.height = float(radius), float(height)
        self.P, self.batch, self.steps = int(pool), int(batch), int(steps)
        self.lr, self.lr_min = float(lr), float(lr_min)
        self.near, self.reach = float(near), float(reach)
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.gen = torch.Generator(device=dev)
        self.gen.manual_seed(seed)
        self.step = 0
        self.next = 0
        self.seed = seed
        # an empty room: every label is the single human's field
        self.empty_ssq = torch.full(grid.shape_zyx, 2 ** 31 - 1,
                                    dtype=torch.int32, device=dev)
        self.xy = np.zeros((self.P, 1, 2), np.float64)
        for p in range(self.P):
            self.xy[p, 0] = self._draw_position()
        self.net = Mlp(n_in=NIN)
        self.loss = torch.zeros(1, device=dev)
        self.in_offset = self.in_scale = None
        self.hist = []

    # -- inputs ----------------------------------------------------------
    def _draw_position(self):
        """A human whose voxelised disk lies wholly inside the grid."""
        g, r = self.grid, self.radius
        lo = np.array(g.origin[:2]) + r + 1.5 * g.h
        hi = np.array(g.origin[:2]) + np.array(g.extent[:2]) - r - 1.5 * g.h
        return self.rng.uniform(lo, hi)

    def _centres(self, n):
        """Centres around the pool's humans: a fraction `near` within
        `reach` metres of the axis (horizontally, at least 2 voxels off the
        disk), the rest uniform over the span of voxel centres; heights
        uniform.  Returns (centre [n, 3], pool index [n]) on the device."""
        import torch
        g, dev, gen = self.grid, self.dev, self.gen
        o = torch.tensor(g.origin, dtype=torch.float64, device=dev)
        L = torch.tensor(g.extent, dtype=torch.float64, device=dev)
        lo, hi = o + g.h / 2, o + L - g.h / 2
        cfg = torch.randint(0, self.P, (n,), generator=gen, device=dev)
        u = torch.rand((n, 4), generator=gen, device=dev,
                       dtype=torch.float64)
        c = lo + u[:, :3] * (hi - lo)
        m = int(n * self.near)
        if m:
            ax = torch.from_numpy(self.xy[:, 0]).to(dev)[cfg[:m]]
            r0 = self.radius + 2 * g.h
            rho = r0 + u[:m, 3] * self.reach
            th = u[:m, 0] * (2 * math.pi)
            c[:m, 0] = ax[:, 0] + rho * torch.cos(th)
            c[:m, 1] = ax[:, 1] + rho * torch.sin(th)
        c = torch.minimum(torch.maximum(c, lo), hi)
        return c.to(torch.float32).contiguous(), cfg.to(torch.int32)

    def batch_rows(self, n):
        """(rows [n, 16], residual targets [n]) of one batch."""
        import torch
        c, cfg = self._centres(n)
        zero = torch.zeros(n, dtype=torch.float32, device=self.dev)
        lab, _, _, _ = query_spheres_direct(
            self.grid, self.empty_ssq, self.xy, self.radius, self.height,
            c, zero, cfg, want_status=False)
        x, _, t = surrogate_human_features(
            self.grid, self.xy, self.radius, self.height, c, cfg,
            label=lab)
        return x, t

    # -- optimisation ----------------------------------------------------
    def init_network(self):
        """Parameters drawn on the host; the input normalisation from the
        statistics of one batch (mean and spread of every feature)."""
        x, _ = self.batch_rows(self.batch)
        xs = x.double()
        off = xs.mean(0).cpu().numpy()
        sd = xs.std(0).cpu().numpy()
        self.in_offset = off.astype(np.float32)
        self.in_scale = (1.0 / np.maximum(sd, 1e-3)).astype(np.float32)
        self.net.set_params(init_params(self.rng, NIN), self.in_offset,
                            self.in_scale, 1.0)

    def lr_at(self, step):
        return self.lr_min + 0.5 * (self.lr - self.lr_min) * (
            1 + math.cos(math.pi * step / self.steps))

    def run(self, until=None, log=print, log_every=1000):
        """Steps up to `until` (default: all), one pool refresh each."""
        until = self.steps if until is None else min(until, self.steps)
        t0 = time.time()
        while self.step < until:
            self.step += 1
            self.xy[self.next, 0] = self._draw_position()
            self.next = (self.next + 1) % self.P
            x, t = self.batch_rows(self.batch)
            self.net.train_step(x, t, self.lr_at(self.step), loss=self.loss)
            if self.step % log_every == 0 or self.step == self.steps:
                l = float(self.loss.cpu()[0])
                if not math.isfinite(l):
                    raise FloatingPointError(f"loss {l} at {self.step}")
                self.hist.append((self.step, l))
                log(json.dumps({"step": self.step, "loss": l,
                                "lr": self.lr_at(self.step),
                                "s": round(time.time() - t0, 1)}))

    # -- checkpoints -----------------------------------------------------
    def save_checkpoint(self, path):
        p, m1, m2, step = self.net.get_state()
        assert step == self.step
        g = self.grid
        meta = {"step": self.step, "steps": self.steps, "next": self.next,
                "P": self.P, "batch": self.batch, "lr": self.lr,
                "lr_min": self.lr_min, "near": self.near,
                "reach": self.reach, "seed": self.seed,
                "radius": self.radius, "height": self.height,
                "grid": [g.nx, g.ny, g.nz], "voxel_m": g.h,
                "origin": list(g.origin), "hist": self.hist,
                "rng": self.rng.bit_generator.state}
        np.savez(path, params=p, m1=m1, m2=m2, in_offset=self.in_offset,
                 in_scale=self.in_scale, pool_xy=self.xy,
                 gen_state=self.gen.get_state().numpy(),
                 meta=json.dumps(meta))

    @classmethod
    def resume(cls, path, grid, dev):
        import torch
        d = np.load(path, allow_pickle=False)
        meta = json.loads(str(d["meta"]))
        if [grid.nx, grid.ny, grid.nz] != meta["grid"] or \
                grid.h != meta["voxel_m"]:
            raise ValueError("checkpoint of another grid")
        t = cls(grid, dev, meta["radius"], meta["height"], meta["P"],
                meta["batch"], meta["steps"], meta["lr"], meta["lr_min"],
                meta["seed"], meta["near"], meta["reach"])
        t.rng.bit_generator.state = meta["rng"]
        t.gen.set_state(torch.from_numpy(d["gen_state"].copy()))
        t.xy = d["pool_xy"].astype(np.float64).copy()
        t.step, t.next, t.hist = meta["step"], meta["next"], meta["hist"]
        t.in_offset = d["in_offset"].astype(np.float32)
        t.in_scale = d["in_scale"].astype(np.float32)
        t.net.set_state(d["params"], d["m1"], d["m2"], meta["step"],
                        t.in_offset, t.in_scale, 1.0)
        return t

    def info(self):
        g = self.grid
        return {"features": FEATURES, "grid": [g.nx, g.ny, g.nz],
                "voxel_m": g.h, "radius_m": self.radius,
                "height_m": self.height, "steps": self.step,
                "batch": self.batch, "samples": self.step * self.batch,
                "pool": self.P, "lr": self.lr, "near": self.near,
                "reach": self.reach,
                "final_loss": self.hist[-1][1] if self.hist else None}


def save(path, trainer, extra=None):
    info = trainer.info()
    if extra:
        info.update(extra)
    np.savez(path, params=trainer.net.get_params(),
             in_offset=trainer.in_offset, in_scale=trainer.in_scale,
             out_scale=np.float32(1.0), meta=json.dumps(info))


def load(path, handle=None):
    """(network, meta dict) from a file written by save()."""
    d = np.load(path, allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    if meta.get("features") != FEATURES:
        raise ValueError(
            f"{path}: weights trained on row transform "
            f"{meta.get('features')!r}, this library computes {FEATURES!r}")
    net = Mlp(handle or default_handle(), n_in=NIN)
    net.set_params(d["params"], d["in_offset"], d["in_scale"],
                   float(d["out_scale"]))
    return net, meta


def _time_ms(fn, reps=5, warmup=2):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def evaluation_scene(name: str, seed: int = 40, n_queries: int = 1_000_000):
    """The evaluation workload of a room: room256 with three fresh
    constant-velocity humans (seed 40) and n_queries spheres (centres
    uniform over the span of voxel centres, radius U(0.05, 0.15) m, slices
    uniform); room512 with its own eight piecewise-linear humans and its
    100k spheres per slice."""
    if name == "room512":
        return scenegen.room512()
    sc = scenegen.room256(n_queries=0)
    rng = np.random.Generator(np.random.PCG64(seed))
    start, vel = scenegen._cv_humans(rng, sc.grid, 3, sc.radius)
    sc.human_xy = scenegen.cv_positions(start, vel, sc.n_slices, sc.dt)
    sc.queries = scenegen.draw_queries(rng, sc.grid, n_queries, sc.n_slices,
                                       slice_mode="uniform")
    return sc


def evaluate(net, sc, dev, margin=0.10, band=None, e2e_queries=10_000):
    """Surrogate vs exact sphere queries on the scene's own queries.

    Errors are measured on the queries the surrogate answers (exact
    answers have no error): max, p99 and mean absolute distance error in
    metres, and the fallback fraction.  Timings by GPU events on the
    stream: the whole surrogate call, its network part (the rows it
    evaluates) and the exact direct queries (planes of every slice built
    inside the call), at the scene's query count and at e2e_queries."""
    import torch

    from . import Handle, _native
    g = sc.grid
    band = 2.0 * math.sqrt(3.0) * g.h if band is None else band
    occ = torch.from_numpy(sc.occ.astype(np.uint8)).to(dev)
    h = net.h
    ssq, sdf = build_static_sdf(g, occ, handle=h)
    del occ
    q = sc.queries
    c = torch.from_numpy(q.centre).to(dev)
    r = torch.from_numpy(q.radius).to(dev)
    s = torch.from_numpy(q.slice).to(dev)

    def direct(cc=c, rr=r, ss=s):
        return query_spheres_direct(g, ssq, sc.human_xy, sc.radius,
                                    sc.height, cc, rr, ss,
                                    want_status=False, handle=h)

    def sur(cc=c, rr=r, ss=s, rows=False):
        return query_spheres_surrogate(
            net, g, ssq, sdf, sc.human_xy, sc.radius, sc.height, cc, rr, ss,
            fallback_margin=margin, band=band, want_status=False,
            want_rows=rows)
    d_ex, g_ex, _, _ = direct()
    out = sur(rows=True)
    torch.cuda.synchronize()
    rows = int(out["rows"].cpu()[0])
    used = out["used_fallback"].bool()
    acc = ~used
    err = (out["dist"] - d_ex).abs()[acc].double().cpu().numpy()
    gerr = (out["grad"] - g_ex).norm(dim=1)[acc].double().cpu().numpy()
    n = len(q.radius)
    res = {"room": sc.name, "queries": n, "humans": sc.n_humans,
           "network_rows": rows, "rows_per_query": rows / n,
           "slices": sc.n_slices, "margin_m": margin, "band_m": band,
           "rule": "fallback when the predicted sphere distance is below "
                   "the margin, the two nearest candidates are within the "
                   "band, or a clipped human comes within the band",
           "fallback_fraction": float(used.float().mean()),
           "err_max_m": float(err.max()) if err.size else None,
           "err_p99_m": float(np.percentile(err, 99)) if err.size else None,
           "err_p999_m": float(np.percentile(err, 99.9)) if err.size
           else None,
           "err_mean_m": float(err.mean()) if err.size else None,
           "grad_err_mean": float(gerr.mean()) if gerr.size else None,
           "grad_err_p99": float(np.percentile(gerr, 99)) if gerr.size
           else None}
    # GPU time of the calls and of the network inside the surrogate call
    h.profile(True, only=[_native.KERNEL_MLP])
    h.profile_reset()
    res["surrogate_path_ms"] = _time_ms(sur)
    mlp_ms, mlp_n = h.profile_read(_native.KERNEL_MLP)
    res["surrogate_network_ms"] = mlp_ms / max(mlp_n, 1)
    # one row: the forward pass (16 -> 4 x 128 -> 1) and the reverse pass
    # to the 16 inputs
    flop = 2 * (16 * 128 + 3 * 128 * 128 + 128) + \
        2 * (3 * 128 * 128 + 16 * 128)
    res["network_flop_per_row"] = flop
    if res["surrogate_network_ms"] > 0:
        res["network_tflops"] = (flop * rows /
                                 (res["surrogate_network_ms"] / 1e3) / 1e12)
        res["network_frac_bf16_peak"] = res["network_tflops"] / 2500.0
    h.profile(False)
    res["exact_direct_ms"] = _time_ms(direct)
    m = min(e2e_queries, n)
    cq, rq, sq = c[:m].contiguous(), r[:m].contiguous(), s[:m].contiguous()
    res["e2e_queries"] = m
    res["e2e_surrogate_ms"] = _time_ms(lambda: sur(cq, rq, sq))
    res["e2e_exact_direct_ms"] = _time_ms(lambda: direct(cq, rq, sq))
    return res


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--room", choices=sorted(ROOMS), default="room256")
    ap.add_argument("--out", required=True)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--batch", type=int, default=32768)
    ap.add_argument("--pool", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--near", type=float, default=0.6)
    ap.add_argument("--reach", type=float, default=1.5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--checkpoint", default="",
                    help="write a checkpoint here every --every steps")
    ap.add_argument("--every", type=int, default=5000)
    ap.add_argument("--resume", default="", help="continue a checkpoint")
    ap.add_argument("--eval", action="store_true",
                    help="evaluate the trained network on the room's "
                         "evaluation workload")
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    grid = room_grid(a.room).grid
    if a.resume:
        t = Trainer.resume(a.resume, grid, dev)
    else:
        t = Trainer(grid, dev, pool=a.pool, batch=a.batch, steps=a.steps,
                    lr=a.lr, seed=a.seed, near=a.near, reach=a.reach)
        t.init_network()
    t0 = time.time()
    while t.step < t.steps:
        t.run(until=t.step + a.every, log=lambda s: print(s, flush=True))
        if a.checkpoint:
            t.save_checkpoint(a.checkpoint)
    save(a.out, t, {"room": a.room, "seconds": round(time.time() - t0, 1)})
    print(json.dumps({"saved": a.out, **t.info()}), flush=True)
    if a.eval:
        sc = evaluation_scene(a.room)
        print(json.dumps({"eval": evaluate(t.net, sc, dev)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

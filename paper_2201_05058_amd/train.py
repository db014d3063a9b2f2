"""Trainer of the sphere-query surrogate for one static room.

Each step of the data pipeline and of the optimisation runs in the
library's kernels.  A pool of P draws of three constant-velocity humans is
kept on the device with the exact fields of all their slices
(pcsdf_predicted_composite_sdf); every step replaces one draw, labels a
batch of sphere centres drawn over all configurations and slices with the
exact distance at the centre (pcsdf_query_spheres with zero radius),
assembles the network input on the device
(pcsdf_surrogate_features_pool) and takes one Adam step on the squared
error (pcsdf_mlp_train_step).  Mixing many configurations in every batch
matters: batches of a single configuration teach the network that
configuration's field, not its dependence on the humans' state.  This module only draws the random inputs
(human starts and velocities on the host, centres and slices with a seeded
torch generator on the device) and sequences the calls.

Two modes.  "env" (the default) trains the network on the humans' part of
the field only -- the exact per-slice field of the cylinders, built by the
same composite call over an empty environment -- and answers queries with
the smaller of the network's value and the environment field sampled
exactly at the centre (the environment field is built once per room, not
per slice).  "pure" trains the network on the full composite; it then has
to memorise the room through its training data, and one network serves
one static room.  Labels below -0.1 m are raised to -0.1 m: deep inside
obstacles the surrogate is never trusted (the fallback rule sends every
predicted distance under the margin to the exact path).  In the env mode
labels are capped 0.2 m above the room's largest environment distance
(there the environment wins the min anyway; the humans' part is +inf when
every human has left the grid).  A fraction of the training centres can be
drawn near the humans (within 1 m of a human's predicted position in x, y),
where the humans' part decides the answer.

Usage:  python -m paper_2201_05058_amd.train --out weights.npz
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

import scenegen

from . import (build_static_sdf, default_handle, predicted_composite_sdf,
               query_spheres, query_spheres_direct)
from .surrogate import (NIN, Mlp, init_params, surrogate_features,
                        surrogate_features_pool)

LABEL_FLOOR = -0.1
# Labels of the env mode are capped just above the room's largest
# environment distance: beyond it the environment always wins the min, and
# the humans' part (+inf where every human has left the grid) stays finite.
CAP_ABOVE_ENV = 0.2


# Name of the network's input transform (the features kernels): weights
# trained on another transform are refused by load().
FEATURES = "axis-offsets-v1"


def normalisation(grid):
    """Input offset/scale bringing the features to about unit range.
    Feature order: centre x y z, t, then per human the offset (dx, dy) from
    its axis at t to the centre, the distance rho to that axis, its
    velocity (vx, vy) and a zero slot."""
    L = np.array(grid.extent, np.float64)
    o = np.array(grid.origin, np.float64)
    D = float(np.hypot(L[0], L[1]))
    off = np.zeros(NIN, np.float64)
    scl = np.ones(NIN, np.float64)
    off[0:3] = o + L / 2
    scl[0:3] = 2.0 / L
    off[3], scl[3] = 1.0, 1.0
    for k in range(3):
        b = 4 + 6 * k
        scl[b:b + 2] = 1.0 / L[:2]
        off[b + 2], scl[b + 2] = D / 2, 2.0 / D
        scl[b + 3:b + 5] = 1.0 / 1.5
    return off.astype(np.float32), scl.astype(np.float32)


MODES = ("env", "pure")


class Room:
    """A static room (occupancy, static field) and the slice schedule."""

    def __init__(self, scene, dev, mode="env"):
        import torch
        if mode not in MODES:
            raise ValueError(f"mode must be one of {MODES}")
        self.sc = scene
        self.grid = scene.grid
        self.dev = dev
        self.mode = mode
        occ = torch.from_numpy(scene.occ.astype(np.uint8)).to(dev)
        self.static_ssq, self.static_sdf = build_static_sdf(self.grid, occ)
        # labels of the env mode: the humans' field over an empty room
        self.empty_ssq = torch.full(self.grid.shape_zyx, 2 ** 31 - 1,
                                    dtype=torch.int32, device=dev)
        self.n_slices = scene.n_slices
        self.dt = scene.dt
        self.fields = torch.empty((self.n_slices,) + self.grid.shape_zyx,
                                  dtype=torch.float32, device=dev)
        fin = self.static_sdf[torch.isfinite(self.static_sdf)]
        self.cap = (float(fin.max()) + CAP_ABOVE_ENV if mode == "env"
                    and fin.numel() else float("inf"))

    def draw_humans(self, rng):
        start, vel = scenegen._cv_humans(rng, self.grid, 3,
                                         scenegen.HUMAN_RADIUS)
        xy = scenegen.cv_positions(start, vel, self.n_slices, self.dt)
        return xy, scenegen.human_state(start, vel)

    def build(self, xy):
        """The exact composite fields of every slice."""
        predicted_composite_sdf(self.grid, self.static_ssq, xy,
                                scenegen.HUMAN_RADIUS, scenegen.HUMAN_HEIGHT,
                                out_sdf=self.fields, want_ssq=False)

    @property
    def label_static(self):
        """The environment the training labels are composited with."""
        return self.empty_ssq if self.mode == "env" else self.static_ssq

    @property
    def env_sdf(self):
        return self.static_sdf if self.mode == "env" else None

    def draw_queries(self, gen, n):
        """Centres uniform over the span of voxel centres, slices uniform."""
        import torch
        g = self.grid
        lo = torch.tensor(np.array(g.origin) + g.h / 2, dtype=torch.float32,
                          device=self.dev)
        span = torch.tensor(np.array(g.extent) - g.h, dtype=torch.float32,
                            device=self.dev)
        c = torch.rand((n, 3), generator=gen, device=self.dev) * span + lo
        s = torch.randint(0, self.n_slices, (n,), generator=gen,
                          device=self.dev, dtype=torch.int32)
        return c.contiguous(), s


class Pool:
    """Label fields of P human configurations at once, so that every
    training batch mixes many configurations: pool slice c*n + s is slice s
    of configuration c.  One configuration is replaced by a fresh draw per
    refresh."""

    def __init__(self, room, P, rng):
        import torch
        self.room, self.P, self.rng = room, P, rng
        n = room.n_slices
        self.fields = torch.empty((P * n,) + room.grid.shape_zyx,
                                  dtype=torch.float32, device=room.dev)
        self.states = torch.zeros((P, NIN - 4), dtype=torch.float32,
                                  device=room.dev)
        self.xy = torch.zeros((P, n, 3, 2), dtype=torch.float32,
                              device=room.dev)
        self.next = 0
        for _ in range(P):
            self.refresh()

    def refresh(self):
        import torch
        room, p = self.room, self.next
        n = room.n_slices
        xy, state = room.draw_humans(self.rng)
        predicted_composite_sdf(room.grid, room.label_static, xy,
                                scenegen.HUMAN_RADIUS, scenegen.HUMAN_HEIGHT,
                                out_sdf=self.fields[p * n:(p + 1) * n],
                                want_ssq=False)
        self.states[p] = torch.from_numpy(state).to(room.dev)
        self.xy[p] = torch.from_numpy(xy.astype(np.float32)).to(room.dev)
        self.next = (p + 1) % self.P

    def batch(self, gen, n, near):
        """(features [n, 22], labels [n]): centres uniform over the span of
        voxel centres (a fraction `near` within 1 m in x, y of a random
        human of the sample's configuration and slice), configurations and
        slices uniform."""
        import torch
        room = self.room
        c, s = room.draw_queries(gen, n)
        cfg = torch.randint(0, self.P, (n,), generator=gen, device=room.dev)
        m = int(n * near)
        if m > 0:
            k = torch.randint(0, 3, (m,), generator=gen, device=room.dev)
            p = self.xy[cfg[:m], s[:m].long(), k]
            off = torch.rand((m, 2), generator=gen, device=room.dev) * 2 - 1
            g = room.grid
            lo = torch.tensor(np.array(g.origin[:2]) + g.h / 2,
                              dtype=torch.float32, device=room.dev)
            hi = torch.tensor(np.array(g.origin[:2]) + np.array(g.extent[:2])
                              - g.h / 2, dtype=torch.float32,
                              device=room.dev)
            c[:m, :2] = torch.minimum(torch.maximum(p + off, lo), hi)
        gs = (cfg.to(torch.int32) * room.n_slices + s).contiguous()
        zero = torch.zeros(n, dtype=torch.float32, device=room.dev)
        d, _, _, _ = query_spheres(room.grid, self.fields, c, zero, gs,
                                   want_status=False)
        y = d.clamp_(min=LABEL_FLOOR, max=room.cap)
        x = surrogate_features_pool(c, gs, room.n_slices, self.P, room.dt,
                                    self.states)
        return x, y


def train(scene, dev, samples=50_000_000, batch=16384, pool=48,
          lr=1e-3, lr_min=1e-5, seed=0, log_every=1000, log=print,
          mode="env", near=0.25):
    import torch
    room = Room(scene, dev, mode)
    rng = np.random.Generator(np.random.PCG64(seed))
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    net = Mlp()
    off, scl = normalisation(room.grid)
    net.set_params(init_params(rng), off, scl, 1.0)
    steps = max(1, samples // batch)
    P = Pool(room, pool, rng)
    loss = torch.zeros(1, device=dev)
    hist = []
    t0 = time.time()
    for step in range(1, steps + 1):
        P.refresh()
        x, y = P.batch(gen, batch, near)
        a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step
                                                         / steps))
        net.train_step(x, y, a, loss=loss)
        if step % log_every == 0 or step == steps:
            l = float(loss.cpu()[0])
            if not math.isfinite(l):
                raise FloatingPointError(f"loss {l} at step {step}")
            hist.append((step, l))
            log(json.dumps({"step": step, "loss": l, "lr": a,
                            "s": round(time.time() - t0, 1)}))
    torch.cuda.synchronize()
    return net, {"steps": steps, "batch": batch, "samples": steps * batch,
                 "seconds": time.time() - t0, "loss": hist,
                 "in_offset": off, "in_scale": scl, "mode": mode,
                 "near": near, "lr": lr, "label_cap": room.cap,
                 "pool": pool}


def save(path, net, info, scene):
    np.savez(path, params=net.get_params(), in_offset=info["in_offset"],
             in_scale=info["in_scale"], out_scale=np.float32(1.0),
             meta=json.dumps({"features": FEATURES,
                              "room": scene.name, "seed": scene.seed,
                              "grid": [scene.grid.nx, scene.grid.ny,
                                       scene.grid.nz],
                              "voxel_m": scene.grid.h,
                              "n_slices": scene.n_slices, "dt": scene.dt,
                              "mode": info["mode"], "near": info["near"],
                              "lr": info["lr"], "pool": info["pool"],
                              "label_cap": info["label_cap"],
                              "samples": info["samples"],
                              "steps": info["steps"],
                              "final_loss": info["loss"][-1][1]
                              if info["loss"] else None}))


def load(path, handle=None):
    """(network, meta dict) from a file written by save()."""
    d = np.load(path, allow_pickle=False)
    meta = json.loads(str(d["meta"]))
    if meta.get("features") != FEATURES:
        raise ValueError(
            f"{path}: weights trained on input transform "
            f"{meta.get('features')!r}, this library computes {FEATURES!r}")
    net = Mlp(handle or default_handle())
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


def evaluate(net, scene, dev, n_queries=1_000_000, seed=40, margin=0.10,
             time_queries=None, mode="env"):
    """Surrogate vs exact sphere queries on a fresh draw of the humans.

    Errors are measured on the queries the surrogate answers (exact
    answers have no error): max, p99 and mean absolute distance error in
    metres, and the fallback fraction.  Timings: the 1M-query call of each
    path on fields already built, and the end-to-end cost per new human
    state at the room's own query load (time_queries, default: the scene's
    query count), where the exact path builds every slice and the surrogate
    path evaluates its fallback queries directly from the chords and the
    static field (as does the direct exact path, timed alongside)."""
    import torch

    from .surrogate import query_spheres_surrogate
    room = Room(scene, dev, mode)
    rng = np.random.Generator(np.random.PCG64(seed))
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    xy, state = room.draw_humans(rng)
    room.build(xy)
    c, s = room.draw_queries(gen, n_queries)
    r = (torch.rand(n_queries, generator=gen, device=dev) * 0.10 + 0.05)
    d_ex, g_ex, _, _ = query_spheres(room.grid, room.fields, c, r, s,
                                     want_status=False)

    def sur(cc=c, rr=r, ss=s):
        return query_spheres_surrogate(
            net, room.grid, room.static_ssq, xy, scenegen.HUMAN_RADIUS,
            scenegen.HUMAN_HEIGHT, state, room.dt, cc, rr, ss,
            fallback_margin=margin, want_status=False,
            static_sdf=room.env_sdf)
    out = sur()
    torch.cuda.synchronize()
    used = out["used_fallback"].bool()
    acc = ~used
    err = (out["dist"] - d_ex).abs()[acc]
    gerr = (out["grad"] - g_ex).norm(dim=1)[acc]
    e = err.double().cpu().numpy()
    ge = gerr.double().cpu().numpy()
    res = {
        "mode": mode, "queries": n_queries, "margin_m": margin,
        "rule": "fallback when predicted sphere distance y - r < margin",
        "fallback_fraction": float(used.float().mean()),
        "err_max_m": float(e.max()) if e.size else None,
        "err_p99_m": float(np.percentile(e, 99)) if e.size else None,
        "err_mean_m": float(e.mean()) if e.size else None,
        "grad_err_mean": float(ge.mean()) if ge.size else None,
        "grad_err_p99": float(np.percentile(ge, 99)) if ge.size else None,
    }
    # kernels at 1M queries on fields already resident
    x = surrogate_features(c, s, room.n_slices, room.dt, state)
    res["mlp_forward_grad_ms_1M"] = _time_ms(lambda: net.forward(x))
    res["exact_query_ms_1M"] = _time_ms(
        lambda: query_spheres(room.grid, room.fields, c, r, s,
                              want_status=False))
    res["surrogate_path_ms_1M"] = _time_ms(sur)
    # end-to-end per new human state at the room's query load
    nq = time_queries or (len(scene.queries.radius) if scene.queries
                          else 10_000)
    cq, sq = c[:nq].contiguous(), (torch.arange(nq, device=dev,
                                                dtype=torch.int32)
                                   % room.n_slices)
    rq = r[:nq].contiguous()

    def exact_e2e():
        room.build(xy)
        query_spheres(room.grid, room.fields, cq, rq, sq, want_status=False)
    def direct(cc, rr, ss):
        return query_spheres_direct(room.grid, room.static_ssq, xy,
                                    scenegen.HUMAN_RADIUS,
                                    scenegen.HUMAN_HEIGHT, cc, rr, ss,
                                    want_status=False)
    res["exact_direct_ms_1M"] = _time_ms(lambda: direct(c, r, s))
    res["e2e_queries"] = nq
    res["e2e_exact_ms"] = _time_ms(exact_e2e)
    res["e2e_exact_direct_ms"] = _time_ms(lambda: direct(cq, rq, sq))
    res["e2e_surrogate_ms"] = _time_ms(lambda: sur(cq, rq, sq))
    o2 = sur(cq, rq, sq)
    used_q = o2["used_fallback"].bool().cpu().numpy()
    res["e2e_fallback_fraction"] = float(used_q.mean())
    res["e2e_slices_with_fallback"] = int(len(np.unique(
        sq.cpu().numpy()[used_q])))
    res["n_slices"] = room.n_slices
    return res


def main(argv=None):
    import torch
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--samples", type=float, default=50e6)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--pool", type=int, default=48,
                    help="human configurations mixed in every batch")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--near", type=float, default=0.25)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--eval", action="store_true",
                    help="evaluate the trained network on 1M queries")
    ap.add_argument("--mode", choices=MODES, default="env")
    a = ap.parse_args(argv)
    dev = torch.device("cuda:0")
    scene = scenegen.room256()
    net, info = train(scene, dev, samples=int(a.samples), batch=a.batch,
                      pool=a.pool, lr=a.lr, seed=a.seed,
                      log=lambda s: print(s, flush=True), mode=a.mode,
                      near=a.near)
    save(a.out, net, info, scene)
    print(json.dumps({"saved": a.out, "samples": info["samples"],
                      "seconds": round(info["seconds"], 1)}), flush=True)
    if a.eval:
        print(json.dumps({"eval": evaluate(net, scene, dev, mode=a.mode)}),
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

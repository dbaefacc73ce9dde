"""Autotuner of the step's launch shape: leaf size, direct-sum tile shape and walk
queue depth, each under an error gate.

The leaf size s is the step's main speed parameter (Sect. 4.2: it moves work between
the direct sums and the expansions without changing the accuracy class).  The direct
sums' tile shape (source moonlets staged per LDS tile, `p2p_tile`, and the most
target moonlets a lane holds, `p2p_targets_max`) and the number of persistent
gravity-walk waves (`walk_waves`: each claims 128 queue items at a time, so this is
the depth of the walk's queue in flight) change how the same work is laid out on the
GPU.  Each is picked by measurement: every candidate runs a few eager steps of the
caller's own workload and the fastest one that passes the gate is kept, one
parameter after the other (s first, then the tile shape at that s, then the walk).

The gate: the RMS relative error of the total acceleration (mutual + central mass)
on sampled moonlets, against the same library's FP64 evaluation with a constant
opening angle of 0.3 at p = 6 (a few 1e-7 on the disks here, more than ten times
below the errors being gated; its lists get room for the extra interactions).  By default a candidate passes when its error is at most twice that
of the configuration the caller starts from (so tuning never trades accuracy for
speed beyond noise); an absolute gate can be given instead.  A candidate above the
gate is chosen only if none passes (then the most accurate one).

Results can be cached in a JSON file keyed by (p, precision, size bucket of N).
Everything here drives the C ABI through the ctypes binding; nothing computes.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = (16, 24, 32, 48, 64, 96, 128)
# (p2p_tile, p2p_targets_max); the first is the library's default
TILE_SHAPES = ((256, 4), (128, 4), (512, 4), (256, 2), (256, 1))
WALK_WAVES = (1024, 512, 2048)
GATE_FACTOR = 2.0


def cache_key(p: int, precision: int, n: int) -> str:
    """N is bucketed by powers of two."""
    return f"p{p}-prec{precision}-n2^{int(math.log2(max(n, 1)))}"


def _copy(nc, prm, **over):
    p2 = nc.Params.from_buffer_copy(prm)
    for k, v in over.items():
        setattr(p2, k, v)
    return p2


def _time_steps(nc, prm, arrays, offsets, dt, steps, device):
    """ms per step of `steps` eager steps after one warm-up step, on copies."""
    import torch
    n = arrays["x"].numel()
    ctx = nc.Context(prm, n, pair_capacity=1 << 16, device=device)
    st = {k: v.clone() for k, v in arrays.items()}
    pairs = torch.zeros((1 << 16, 3), dtype=torch.int64, device=device)
    npairs = torch.zeros(max(steps, 1), dtype=torch.int64, device=device)

    def go(k):
        args = (st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"], st["R"],
                dt, k, pairs, npairs)
        if offsets is None:
            ctx.step(*args)
        else:
            ctx.step_batched(offsets, *args)

    go(1)
    torch.cuda.synchronize()
    ctx.check_status()
    t0 = time.perf_counter()
    go(steps)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    ctx.check_status()
    ctx.close()
    return ms


def _total_accel(nc, prm, arrays, offsets, idx, device):
    """Mutual (the library's gravity under prm) plus central-mass acceleration of the
    moonlets idx at the arrays' state, as a (len(idx), 3) device tensor."""
    import torch
    n = arrays["x"].numel()
    ctx = nc.Context(prm, n, pair_capacity=1 << 10, device=device)
    a = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(3)]
    if offsets is None:
        ctx.build_tree(arrays["x"], arrays["y"], arrays["z"])
    else:
        ctx.build_tree_batched(offsets, arrays["x"], arrays["y"], arrays["z"])
    ctx.gravity(arrays["m"], *a)
    torch.cuda.synchronize()
    ctx.check_status()
    ctx.close()
    r = torch.stack([arrays["x"][idx], arrays["y"][idx], arrays["z"][idx]], 1)
    r3 = torch.linalg.norm(r, dim=1, keepdim=True) ** 3
    return torch.stack([a[0][idx], a[1][idx], a[2][idx]], 1) - prm.G * prm.M_central * r / r3


def _gate_error(acc, ref):
    import torch
    e = torch.linalg.norm(acc - ref, dim=1) / torch.linalg.norm(ref, dim=1)
    return float(torch.sqrt(torch.mean(e * e)).item())


def tune_step(nc, prm, arrays, offsets=None, dt=1e-3, steps=3, leaf_sizes=CANDIDATES,
              tile_shapes=TILE_SHAPES, walk_waves=WALK_WAVES, gate=None,
              samples=4096, seed=12345, device="cuda:0"):
    """Picks leaf_size, then (p2p_tile, p2p_targets_max), then walk_waves for the step
    of `prm` on `arrays` (device tensors x..R; offsets: int64 device tensor of a
    batched call, or None).  gate: the largest error allowed (None: GATE_FACTOR times
    the error of `prm` as given).  Returns (tuned Params, table) where the table
    lists, per stage, every candidate's ms per step, gate error and whether it
    passed."""
    import torch
    n = arrays["x"].numel()
    g = torch.Generator(device="cpu").manual_seed(seed)
    idx = torch.randperm(n, generator=g)[:min(samples, n)].to(device)
    ref_s = 96
    cells = 8 * n // ref_s + 1024
    ref_prm = _copy(nc, prm, p=6, precision=nc.FP64, theta_min=0.3, theta_mode=1,
                    leaf_size=ref_s, p2p_tile=0, p2p_targets_max=0, walk_waves=0,
                    m2l_per_cell=8192, p2p_per_leaf=8192, m2l_capacity=256 * cells,
                    p2p_capacity=128 * cells,
                    queue_capacity=min(100_000_000, 400 * cells))
    ref = _total_accel(nc, ref_prm, arrays, offsets, idx, device)
    start_err = _gate_error(_total_accel(nc, prm, arrays, offsets, idx, device), ref)
    if gate is None:
        gate = GATE_FACTOR * start_err

    def measure(p2):
        err = _gate_error(_total_accel(nc, p2, arrays, offsets, idx, device), ref)
        ms = _time_steps(nc, p2, arrays, offsets, dt, steps, device)
        return {"ms_per_step": ms, "gate_error": err, "passed": bool(err <= gate)}

    def pick(rows):
        ok = {k: v for k, v in rows.items() if v["passed"]}
        pool = ok if ok else rows         # nothing passes: the most accurate one
        key = (lambda k: pool[k]["ms_per_step"]) if ok else (lambda k: pool[k]["gate_error"])
        return min(pool, key=key)

    table = {"gate": gate, "start_error": start_err,
             "gate_metric": "rms relative error of the total acceleration against the "
             "library's FP64 p = 6 evaluation at constant theta = 0.3",
             "samples": int(idx.numel())}
    cur = _copy(nc, prm)
    rows = {}
    for s in leaf_sizes:
        rows[int(s)] = measure(_copy(nc, cur, leaf_size=int(s)))
    cur.leaf_size = int(pick(rows))
    table["leaf_size"] = rows
    rows = {}
    for tile, tmax in tile_shapes:
        rows[f"{tile}x{tmax}"] = measure(_copy(nc, cur, p2p_tile=tile, p2p_targets_max=tmax))
    best = pick(rows)
    cur.p2p_tile, cur.p2p_targets_max = (int(v) for v in best.split("x"))
    table["p2p_tile_x_targets_max"] = rows
    rows = {}
    for w in walk_waves:
        rows[int(w)] = measure(_copy(nc, cur, walk_waves=int(w)))
    cur.walk_waves = int(pick(rows))
    table["walk_waves"] = rows
    table["best"] = {"leaf_size": int(cur.leaf_size), "p2p_tile": int(cur.p2p_tile),
                     "p2p_targets_max": int(cur.p2p_targets_max),
                     "walk_waves": int(cur.walk_waves)}
    return cur, table


def tune_leaf_size(nc, prm, arrays, offsets=None, dt=1e-3, steps=3, candidates=CANDIDATES,
                   cache_path=None, device="cuda:0"):
    """Times `steps` eager steps (after one warm-up step) for every candidate leaf
    size on copies of `arrays` (device tensors x..R); offsets: int64 device tensor
    of a batched call, or None for the plain step.  Returns (best_s, {s: ms/step}).
    No error gate: for callers that only move s."""
    n = arrays["x"].numel()
    key = cache_key(prm.p, prm.precision, n)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cached = json.load(f)
        if key in cached:
            ent = cached[key]
            return int(ent["best"]), {int(k): v for k, v in ent["ms_per_step"].items()}
    table = {}
    for s in candidates:
        table[int(s)] = _time_steps(nc, _copy(nc, prm, leaf_size=int(s)), arrays, offsets, dt,
                                    steps, device)
    best = min(table, key=table.get)
    if cache_path:
        cached = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cached = json.load(f)
        cached[key] = {"best": best, "ms_per_step": table}
        with open(cache_path, "w") as f:
            json.dump(cached, f, indent=1, sort_keys=True)
    return best, table

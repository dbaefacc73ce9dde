"""Leaf-size autotuner for the batched and plain steps.

The leaf size s is the step's main speed parameter (Sect. 4.2: it moves work
between the direct sums and the expansions without changing the accuracy class),
so it is picked by measurement: each candidate runs a few eager steps of the
caller's own workload on the GPU and the fastest is kept.  The direct-sum tile
shape needs no tuning pass: the kernel sizes its lane groups from each leaf's
moonlet count at run time.

Results can be cached in a JSON file keyed by (p, precision, size bucket of N).
Everything here drives the C ABI through the ctypes binding; nothing computes.
"""
from __future__ import annotations

import json
import math
import os
import time

CANDIDATES = (16, 24, 32, 48, 64, 96, 128)


def cache_key(p: int, precision: int, n: int) -> str:
    """N is bucketed by powers of two."""
    return f"p{p}-prec{precision}-n2^{int(math.log2(max(n, 1)))}"


def tune_leaf_size(nc, prm, arrays, offsets=None, dt=1e-3, steps=3, candidates=CANDIDATES,
                   cache_path=None, device="cuda:0"):
    """Times `steps` eager steps (after one warm-up step) for every candidate leaf
    size on copies of `arrays` (device tensors x..R); offsets: int64 device tensor
    of a batched call, or None for the plain step.  Returns (best_s, {s: ms/step})."""
    import torch
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
        p2 = nc.Params.from_buffer_copy(prm)
        p2.leaf_size = int(s)
        ctx = nc.Context(p2, n, pair_capacity=1 << 16, device=device)
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
        table[int(s)] = (time.perf_counter() - t0) * 1e3 / steps
        ctx.check_status()
        ctx.close()
        del ctx, st
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

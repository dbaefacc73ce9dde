#!/usr/bin/env python3
"""Throughput of the falcON tree step (gravity + collision search) on one MI355X.

Workload: a cold disk of N = 1e6 moonlets around a central mass of 1 (G = 1),
expansion order p = 6, theta_min = 0.5 with the mass-dependent opening angle,
leaf size 52 and the walk thresholds of the paper's timing runs, dt = 1e-3.  One
step = collision climb + walk + pair tests + elastic resolution of the pairs found
(as in the paper's timing runs), drift, rebuild (keys, sort, octree),
gravity climb + walk + M2L + descent + direct sums + evaluation, kicks (one
ncorp_step call runs all K steps; its extra initial force evaluation is inside
the timed region).  The headline value is the FP32-bulk form; the plain FP64
form is measured the same way and reported beside it.

Beside it (key "batched") the batched form is measured: 64 independent disks of
log-uniform sizes in [1000, 50000] (about 0.8e6 moonlets in all), p = 4,
theta_min = 0.5, FP32-bulk, leaf size picked by the autotuner, all disks stepped
by the same launches, 50 steps captured in one hipGraph and replayed.

Prints one JSON line (see the keys below).  --gpus N > 1 is refused: this build
runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X FP64 vector (published)
FLOPS_PER_INTERACTION = 20  # directed moonlet pair, the usual N-body convention

# HBM traffic of one direct-sum evaluation (k_p2p<float>) on the
# default workload: FETCH_SIZE and WRITE_SIZE from two rocprofv3 --pmc runs (KiB per
# dispatch), scaled by what the same counters read for a 1 GiB device copy
# (bench.py --copy-calibration 1024: FETCH 524303 KiB -> x2.00, WRITE 1048576 KiB ->
# x1.00).  The figures belong to the kernel source with this git blob hash and are
# reported only while it is unchanged.
# Measured per leaf size (the direct sums' work depends on it).
P2P_TRAFFIC = {"source": "paper_2310_20374_amd/csrc/p2p.hip",
               "blob": "24806f309f8c8f758dd3293823e9518d4bee879f",
               "fetch_scale": 2.00, "write_scale": 1.00,
               # measured launch shape: (leaf size, source tile, most targets per lane)
               "by_shape": {(96, 256, 4): {"fetch_kib": (198843.8,), "write_kib": (25534.3,)},
                            (96, 128, 4): {"fetch_kib": (197890.7,), "write_kib": (25499.9,)}}}


def _git_blob(path):
    import hashlib
    data = open(path, "rb").read()
    return hashlib.sha1(b"blob %d\0" % len(data) + data).hexdigest()


def _p2p_traffic(args, prm):
    """HBM bytes of one direct-sum launch from the stored counters, when they were taken
    on this source, this workload and this launch shape; else None."""
    t = P2P_TRAFFIC
    default = args.n == 1_000_000 and args.p == 6 and args.theta == 0.5
    shape = (int(prm.leaf_size), int(prm.p2p_tile) or 256, int(prm.p2p_targets_max) or 4)
    m = t["by_shape"].get(shape)
    if not default or m is None or _git_blob(os.path.join(ROOT, t["source"])) != t["blob"]:
        return None
    kib = sum(m["fetch_kib"]) * t["fetch_scale"] + sum(m["write_kib"]) * t["write_scale"]
    return kib * 1024.0


def _run(nc, prm, d, dt, steps, warmup, timing, device):
    import torch
    n = len(d["x"])
    ctx = nc.Context(prm, n, pair_capacity=1 << 20, device=device)
    base = {k: torch.tensor(v, device=device) for k, v in d.items()}
    st = {k: v.clone() for k, v in base.items()}
    pairs = torch.zeros((1 << 20, 3), dtype=torch.int64, device=device)
    npairs = torch.zeros(max(steps, warmup, 1), dtype=torch.int64, device=device)

    def reset():
        for k in st:
            st[k].copy_(base[k])

    def go(k):
        ctx.step(st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"], st["R"], dt,
                 k, pairs, npairs)

    if warmup > 0:
        go(warmup)
        torch.cuda.synchronize()
        ctx.check_status()
    reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    go(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.check_status()
    wall = t1 - t0
    n_pairs = int(npairs[:steps].sum().item())
    phases = None
    info = None
    if timing:
        reset()
        ctx.set_timing(True)
        go(steps)
        torch.cuda.synchronize()
        ctx.check_status()
        phases = ctx.phase_times()
        info = ctx.tree_info()
        ctx.set_timing(False)
    # accelerations at the initial state, for the error check
    reset()
    a = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(3)]
    ctx.build_tree(st["x"], st["y"], st["z"])
    ctx.gravity(st["m"], *a)
    torch.cuda.synchronize()
    ctx.check_status()
    acc = torch.stack(a, 1).cpu().numpy()
    mesh = None
    if prm.gravity_method == nc.GRAVITY_MESH or prm.collision_method == nc.COLLISIONS_MESH:
        mesh = ctx.mesh_state()
    return {"wall_s": wall, "phases": phases, "info": info, "acc": acc, "pairs": n_pairs,
            "mesh": mesh}


def _gravity_method_comparison(nc, d, p_list, reps, device, falcon_leaf=None):
    """One tree build plus one gravity evaluation by falcON (Alg. 2, default thresholds,
    FP64, leaf size falcon_leaf: the main line's FP64 leaf size; the order's default
    when None) and by the standard tree code (Alg. 1, leaf size 102, N_cb,pre 6,
    N_cb,post 16: the settings of the paper's speed comparison), at each order in
    p_list; then a collision search (dt = 1e-3) by each on its own tree."""
    import torch
    n = len(d["x"])
    t = {k: torch.tensor(d[k], device=device) for k in ("x", "y", "z", "m", "vx", "vy", "vz",
                                                        "R")}
    a = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(3)]
    pairs = torch.zeros((1 << 16, 2), dtype=torch.int64, device=device)
    npairs = torch.zeros(1, dtype=torch.int64, device=device)
    out = {}
    for p in p_list:
        fprm = (nc.params_default(p) if falcon_leaf is None
                else nc.params_default(p, leaf_size=int(falcon_leaf)))
        for name, prm in (("falcon", fprm),
                          ("standard_tree", nc.params_default(
                              p, leaf_size=102, gravity_method=nc.GRAVITY_STANDARD_TREE,
                              collision_method=nc.COLLISIONS_STANDARD_TREE,
                              ncb_pre=6, ncb_post=16))):
            ctx = nc.Context(prm, n, pair_capacity=1 << 16, device=device)

            def once():
                ctx.build_tree(t["x"], t["y"], t["z"])
                ctx.gravity(t["m"], *a)

            once()
            torch.cuda.synchronize()
            ctx.check_status()
            t0 = time.perf_counter()
            for _ in range(reps):
                once()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / reps
            ctx.check_status()
            # collision search on the same tree (falcON: from the gravity walk's lists)
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.collide(t["vx"], t["vy"], t["vz"], t["R"], 1e-3, pairs, npairs)
            torch.cuda.synchronize()
            ms_col = (time.perf_counter() - t0) * 1e3 / reps
            ctx.check_status()
            n_pairs = int(npairs.item())
            ctx.set_timing(True)
            once()
            torch.cuda.synchronize()
            ph = {k: round(v[0], 4) for k, v in ctx.phase_times().items() if v[1] > 0}
            out[f"{name}_p{p}"] = {"ms_tree_and_gravity": ms, "ms_collision_search": ms_col,
                                   "collision_pairs": n_pairs, "phases_ms": ph,
                                   "leaf_size": prm.leaf_size,
                                   "acc": torch.stack(a, 1).cpu().numpy()}
            del ctx
    return out


def _run_mesh(nc, d, args, device):
    """The mesh module (Sect. 3.3) for both gravity and collisions on the same disk and
    step loop: x = 8 neighbours, Eq. (4) with h/r = 0.05 at the first mesh, Eq. (6)
    after; elastic resolution as in the main line."""
    cmode = nc.COLLISIONS_RESOLVE if args.collisions == "resolve" else nc.COLLISIONS_REPORT
    prm = nc.params_default(args.p, gravity_method=nc.GRAVITY_MESH,
                            collision_method=nc.COLLISIONS_MESH, mesh_neighbours=8.0,
                            mesh_aspect=0.05, mesh_cells=256, collision_mode=cmode,
                            collision_f=2.0)
    r = _run(nc, prm, d, args.dt, args.steps, args.warmup, True, device)
    out = {"ms_per_step": r["wall_s"] * 1e3 / args.steps,
           "value": len(d["x"]) * args.steps / r["wall_s"],
           "phases_ms_per_step": {k: round(v[0] / args.steps, 4)
                                  for k, v in r["phases"].items() if v[1] > 0},
           "collision_pairs_in_timed_steps": r["pairs"], "mesh": r.get("mesh"),
           "mesh_cells": prm.mesh_cells, "neighbours_target": prm.mesh_neighbours}
    return out, r["acc"]


_DIRECT = {}


def _errors(orc, d, acc, samples):
    import numpy as np
    from paper_2310_20374_amd import inputs
    tg = inputs.sample_targets(len(d["x"]), samples)
    key = (id(d), samples)
    if key not in _DIRECT:          # the FP64 direct sums of one input, computed once
        _DIRECT[key] = (orc.direct_sum(d["x"], d["y"], d["z"], d["m"], targets=tg),
                        orc.central_accel(d["x"][tg], d["y"][tg], d["z"][tg]))
    ad, ac = _DIRECT[key]

    def stats(a, ref):
        e = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
        return float(np.sqrt(np.mean(e * e))), float(e.max()), float(np.median(e))

    def scalar_median(a, ref):
        # the paper's measure (Fig. 4): |a - a_ref| / a_ref of the scalar accelerations
        na, nr = np.linalg.norm(a, axis=1), np.linalg.norm(ref, axis=1)
        return float(np.median(np.abs(na - nr) / nr))

    tot = stats(acc[tg] + ac, ad + ac)
    mut = stats(acc[tg], ad)
    return {"rms_total": tot[0], "max_total": tot[1], "median_total": tot[2],
            "rms_mutual": mut[0], "max_mutual": mut[1], "median_mutual": mut[2],
            "scalar_median_total": scalar_median(acc[tg] + ac, ad + ac),
            "scalar_median_mutual": scalar_median(acc[tg], ad),
            "samples": int(len(tg))}


# leaf sizes the main line's autotuner tries (FP64 direct sums cost twice as much, so
# its optimum sits lower)
LEAF_CANDIDATES_FP32 = (52, 64, 80, 96, 112, 128)
LEAF_CANDIDATES_FP64 = (40, 52, 64, 80, 96)

PEAK_HBM_GBS = 8000.0      # MI355X HBM3E (published)


def _phase_rooflines(phases, info, n, p, precision_fp32):
    """Roofline time per phase call from its algorithmic traffic or arithmetic (lower
    bounds: each array read or written once, the paper's operation counts), against
    the phase's measured time per call.  The walks are latency-bound and have no
    roofline; the step's fraction is the sum of roofline times over the sum of the
    measured times of all phases."""
    nm = {0: 0, 1: 1}.get(p, p * (p + 1) * (p + 2) // 6 - 3)
    nl = (p + 1) * (p + 2) * (p + 3) // 6 - 1 if p > 0 else 0
    cells, leaves = info["ncells"], info["nleaves"]
    fpeak = (PEAK_FP32_TFLOPS if precision_fp32 else PEAK_FP64_TFLOPS) * 1e12
    hbm = PEAK_HBM_GBS * 1e9
    m2l_flops = {6: 1650, 5: 1000, 4: 536, 3: 194, 2: 60, 1: 20}.get(p, 0)
    model = {
        "keys": ("hbm", 36.0 * n / hbm, "read x, y, z; write key, index"),
        "sort": ("hbm", 24.0 * n / hbm, "read and write (key, index) once"),
        "tree": ("hbm", (52.0 * n + 8.0 * n + 64.0 * cells) / hbm,
                 "gather positions (read, write, index); read keys; write cell records"),
        "gclimb": ("hbm", (20.0 * n + 32.0 * n + (8.0 * nm + 56.0) * cells) / hbm,
                   "gather masses; read positions and masses once; write moments and cell data"),
        "m2l": ("valu", m2l_flops * info["m2l_dir"] / fpeak,
                "D tensors and the Eq. (25) contraction per directed interaction"),
        "descent": ("hbm", (8.0 * nl * (cells + leaves)) / hbm,
                    "read every cell's C once, write every leaf's"),
        "p2p": ("valu", FLOPS_PER_INTERACTION * info["p2p_inter"] / fpeak,
                "20 flop per directed moonlet pair"),
        "l2p": ("hbm", (72.0 * n + 8.0 * nl * leaves) / hbm,
                "read positions and direct sums, leaf C; write accelerations"),
        "collide": ("hbm+valu", (124.0 * n) / hbm + 10.0 * info["col_tests"] / (PEAK_FP64_TFLOPS * 1e12),
                    "gather velocities and radii, read positions; 10 flop per moonlet pair "
                    "examined (distance against the reaches; Eqs. 1-2 only within reach)"),
        "integrate": ("hbm", 84.0 * n / hbm, "a kick or a drift: about 84 B per moonlet"),
    }
    out, roof_sum, meas_sum = {}, 0.0, 0.0
    for ph, (ms, cnt) in phases.items():
        if cnt <= 0:
            continue
        per_call = ms / cnt / 1e3
        meas_sum += ms
        if ph not in model:
            out[ph] = {"bound": "latency", "ms_per_call": per_call * 1e3}
            continue
        bound, t, basis = model[ph]
        roof_sum += t * cnt * 1e3
        out[ph] = {"bound": bound, "ms_per_call": per_call * 1e3, "roof_ms_per_call": t * 1e3,
                   "frac": t / per_call if per_call > 0 else None, "basis": basis}
    return out, (roof_sum / meas_sum if meas_sum > 0 else None)


def _run_batched(nc, args, device):
    """The batched form: autotuned leaf size, then a 50-step ncorp_step_batched call
    captured in a hipGraph and replayed (the state keeps evolving across replays)."""
    import numpy as np
    import torch
    from paper_2310_20374_amd import autotune, inputs
    sizes = inputs.batch_sizes(64, seed=0)
    d, off = inputs.disk_batch(sizes)
    n = len(d["x"])
    base = {k: torch.tensor(v, device=device) for k, v in d.items()}
    offd = torch.tensor(off, device=device)
    prm = nc.params_default(4, theta_min=0.5, precision=nc.FP32_BULK,
                            collision_mode=nc.COLLISIONS_RESOLVE if args.collisions == "resolve"
                            else nc.COLLISIONS_REPORT, collision_f=2.0)
    t0 = time.perf_counter()
    prm, tuning = autotune.tune_step(nc, prm, base, offd, dt=args.dt, steps=3,
                                     samples=min(args.samples, 2048), device=device)
    tune_s = time.perf_counter() - t0
    best = prm.leaf_size
    table = {s: v["ms_per_step"] for s, v in tuning["leaf_size"].items()}
    ns = args.batched_steps
    ctx = nc.Context(prm, n, pair_capacity=1 << 18, device=device)
    st = {k: v.clone() for k, v in base.items()}
    pairs = torch.zeros((1 << 18, 3), dtype=torch.int64, device=device)
    npairs = torch.zeros(ns, dtype=torch.int64, device=device)

    def go():
        ctx.step_batched(offd, st["x"], st["y"], st["z"], st["vx"], st["vy"], st["vz"], st["m"],
                         st["R"], args.dt, ns, pairs, npairs)

    # eager call: warm-up and the non-graph rate
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    go()
    torch.cuda.synchronize()
    eager_s = time.perf_counter() - t0
    ctx.check_status()
    for k in st:
        st[k].copy_(base[k])
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        go()
    g.replay()                       # warm replay
    torch.cuda.synchronize()
    ctx.check_status()
    t0 = time.perf_counter()
    for _ in range(args.batched_replays):
        g.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.check_status()
    total_steps = ns * args.batched_replays
    # accuracy at the initial state: sampled moonlets against each disk's FP64 direct sum
    errors = None
    if not args.no_errors:
        import oracle as orc
        a = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(3)]
        for k in st:
            st[k].copy_(base[k])
        ctx.build_tree_batched(offd, st["x"], st["y"], st["z"])
        ctx.gravity(st["m"], *a)
        torch.cuda.synchronize()
        ctx.check_status()
        acc = torch.stack(a, 1).cpu().numpy()
        tg = inputs.sample_targets(n, args.samples)
        disk_of = np.searchsorted(off, tg, side="right") - 1
        ad = np.zeros((len(tg), 3))
        for k in np.unique(disk_of):
            sel = disk_of == k
            lo, hi = off[k], off[k + 1]
            ad[sel] = orc.direct_sum(d["x"][lo:hi], d["y"][lo:hi], d["z"][lo:hi], d["m"][lo:hi],
                                     targets=tg[sel] - lo)
        ac = orc.central_accel(d["x"][tg], d["y"][tg], d["z"][tg])

        def stats(x, ref):
            e = np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)
            return float(np.sqrt(np.mean(e * e))), float(e.max())

        rt, mt = stats(acc[tg] + ac, ad + ac)
        rm, mm = stats(acc[tg], ad)
        errors = {"rms_total": rt, "max_total": mt, "rms_mutual": rm, "max_mutual": mm,
                  "samples": int(len(tg))}
    return {
        "workload": "64 independent cold disks (sizes log-uniform in [1000, 50000], seed 0; "
                    "disk k drawn with seed 1000+k), one root per disk, no cross-disk terms",
        "n_disks": 64, "n": int(n), "p": 4, "theta_min": 0.5, "precision": "fp32-bulk",
        "collisions": args.collisions,
        "leaf_size": int(best), "autotune_ms_per_step": table, "autotune_seconds": tune_s,
        "autotune": tuning,
        "graph_steps": ns, "replays": args.batched_replays,
        "value": n * total_steps / wall, "unit": "particle-steps/s",
        "ms_per_step": wall * 1e3 / total_steps,
        "eager_value": n * ns / eager_s, "eager_ms_per_step": eager_s * 1e3 / ns,
        "collision_pairs_per_step": float(npairs.sum().item()) / ns,
        "errors": errors,
    }


def _run_clustered(nc, args, device, leaf_size, cmode):
    """The clustered stress workload: N = 4e6 moonlets, half a cold disk and half in
    200 Plummer clumps (scale 0.05, clump weights dM ~ M^-2 dM), FP32-bulk, p = 6,
    theta_min = 0.5, the main line's FP32-bulk leaf size, collisions resolved as in the
    main line.  Reports the step rate, the pairs per step, the load balance of the last
    gravity evaluation (the gravity walk's per-wave busy clock cycles, max over mean; the
    direct sums' source moonlets per target moonlet, max over mean), and the complete pair
    set of one search on the initial state against the oracle's exact grid scan."""
    import numpy as np
    import torch
    from paper_2310_20374_amd import inputs
    n = args.clustered_n
    d = inputs.clumps(n, seed=0)
    prm = nc.params_default(6, theta_min=args.theta, precision=nc.FP32_BULK,
                            collision_mode=cmode, collision_f=2.0, leaf_size=int(leaf_size))
    steps = args.clustered_steps
    r = _run(nc, prm, d, args.dt, steps, 1, True, device)
    info = r["info"]
    ph = r["phases"]
    out = {"workload": "clustered: half a cold disk, half in 200 Plummer clumps "
                       "(scale 0.05), FP32-bulk",
           "n": n, "p": 6, "theta_min": args.theta, "leaf_size": int(leaf_size),
           "steps": steps, "ms_per_step": r["wall_s"] * 1e3 / steps,
           "particle_steps_per_s": n * steps / r["wall_s"],
           "pairs_per_step": r["pairs"] / steps,
           "phases_ms_per_step": {k: round(v[0] / steps, 4) for k, v in ph.items()},
           "tree": {k: info[k] for k in ("ncells", "nleaves", "maxlevel", "m2l", "p2p",
                                         "visited", "p2p_inter", "m2l_maxlist",
                                         "p2p_maxlist")},
           "load_balance": {
               "walk_busy_cycles_max": info["walk_busy_max"],
               "walk_busy_cycles_mean": info["walk_busy_mean"],
               "walk_busy_max_over_mean": info["walk_busy_max"] / max(info["walk_busy_mean"], 1),
               "direct_sum_sources_max": info["p2p_src_max"],
               "direct_sum_sources_mean": info["p2p_inter"] / n,
               "direct_sum_sources_max_over_mean": info["p2p_src_max"] * n / max(
                   info["p2p_inter"], 1),
               "m2l_list_max": info["m2l_maxlist"],
               "m2l_list_mean": info["m2l_dir"] / max(info["ncells"], 1)}}
    # the complete pair set of one search on the seeded state, against the oracle
    t = {k: torch.tensor(v, device=device) for k, v in d.items()}
    cap = 1 << 20
    ctx = nc.Context(prm, n, pair_capacity=cap, device=device)
    pairs = torch.zeros((cap, 2), dtype=torch.int64, device=device)
    npairs = torch.zeros(1, dtype=torch.int64, device=device)
    a = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(3)]
    ctx.build_tree(t["x"], t["y"], t["z"])
    ctx.gravity(t["m"], *a)
    ctx.collide(t["vx"], t["vy"], t["vz"], t["R"], args.dt, pairs, npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    k = int(npairs.item())
    got = pairs[:k].cpu().numpy()
    del ctx, t, a, pairs
    out["_d"] = d
    out["_acc"] = r["acc"]
    out["_pairs"] = got
    return out


def _cpu_step(orc, n, p, theta, s, thr, dt):
    """One steady-state step of the oracle as it stands (single-threaded FP64 tree,
    recursive walk, full 3^n tensors) on an N-moonlet cold disk: a tree build and the
    gravity evaluation, then a tree build and the collision walk (the drift and kicks
    are negligible beside them).  Returns (gravity seconds, collision seconds)."""
    from paper_2310_20374_amd import inputs
    d = inputs.disk(n, seed=0)
    t0 = time.perf_counter()
    orc.tree_accel(d, p=p, theta_min=theta, s=s, ncs=thr[0], ncc_pre=thr[1], ncc_post=thr[2])
    t1 = time.perf_counter()
    t = orc.Tree(d["x"], d["y"], d["z"], s)
    orc.Collide(t, d["vx"], d["vy"], d["vz"], d["R"], dt).run(12, 0, 16)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def _cpu_baseline(orc, n_sample, p, theta, s, thr, dt):
    """The oracle timed on one host core for one steady-state step of the headline's
    disk (N = n_sample, same distribution and settings)."""
    g, c = _cpu_step(orc, n_sample, p, theta, s, thr, dt)
    return {"value": n_sample / (g + c), "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"one steady-state step of an N={n_sample} cold disk (same distribution, "
                      f"p={p}, theta_min={theta}, s={s}): tree build + FP64 oracle gravity, "
                      f"tree build + collision walk; single-threaded",
            "seconds": g + c, "gravity_seconds": g, "collision_seconds": c}


def _cpu_configs(orc, dt):
    """The oracle's per-step rate on the two small configurations of the benchmark:
    N = 2000, p = 3, s = 16, and N = 1e5, p = 6 (its default leaf size, s = 52); one
    steady-state step each, single-threaded."""
    out = {}
    for name, n, p, s, thr in (("n2000_p3_fp64", 2000, 3, 16, (64, 8, 64)),
                               ("n100000_p6_fp64", 100_000, 6, 52, (256, 256, 512))):
        g, c = _cpu_step(orc, n, p, 0.5, s, thr, dt)
        out[name] = {"value": n / (g + c), "unit": "particle-steps/s", "cores": 1,
                     "gravity_seconds": g, "collision_seconds": c}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--p", type=int, default=6)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--samples", type=int, default=4096)
    ap.add_argument("--cpu-sample", type=int, default=500_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--fp32-only", action="store_true")
    ap.add_argument("--collisions", choices=("resolve", "report"), default="resolve",
                    help="resolve the pairs found elastically (f = 2, as in the paper's timing "
                         "runs, keeping N constant) or only report them")
    ap.add_argument("--leaf-size", default="auto",
                    help="leaf size s of the main line: 'auto' (the autotuner, each precision "
                         "form on its own) or an integer")
    ap.add_argument("--launch-shape", default="",
                    help="with an integer --leaf-size: 'TILExTMAX:WAVES' pins the direct-sum "
                         "tile shape and the walk's wave count (e.g. 256x4:512); '' keeps the "
                         "library's defaults")
    ap.add_argument("--thetas", default="0.3,0.7",
                    help="extra opening angles timed and error-checked beside --theta "
                         "(both precision forms, 10 steps each); '' for none")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-clustered", action="store_true",
                    help="skip the clustered stress workload (4e6 moonlets, disk + clumps)")
    ap.add_argument("--clustered-n", type=int, default=4_000_000)
    ap.add_argument("--clustered-steps", type=int, default=5)
    ap.add_argument("--no-mesh", action="store_true",
                    help="skip the mesh-module step loop (gravity and collisions on the mesh)")
    ap.add_argument("--no-method-comparison", action="store_true",
                    help="skip the falcON / standard tree comparison (one gravity evaluation "
                         "each at p = 3 and at --p)")
    ap.add_argument("--batched-only", action="store_true",
                    help="measure only the batched form (its object is printed alone)")
    ap.add_argument("--clustered-only", action="store_true",
                    help="measure only the clustered stress workload at --leaf-size (96 when "
                         "'auto'); its object is printed alone")
    ap.add_argument("--batched-steps", type=int, default=50)
    ap.add_argument("--batched-replays", type=int, default=4)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (three times) and exit: the "
                         "reference kernel for scaling the FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes}))
        return 0

    from paper_2310_20374_amd import inputs, ncorp
    device = "cuda:0"
    if args.batched_only:
        print(json.dumps({"batched": _run_batched(ncorp, args, device)}))
        return 0
    cmode = ncorp.COLLISIONS_RESOLVE if args.collisions == "resolve" else ncorp.COLLISIONS_REPORT
    if args.clustered_only:
        s = 96 if args.leaf_size == "auto" else int(args.leaf_size)
        cl = _run_clustered(ncorp, args, device, s, cmode)
        for k in ("_d", "_acc", "_pairs"):    # the error and pair checks need the oracle
            cl.pop(k)
        print(json.dumps({"clustered": cl}))
        return 0
    d = inputs.disk(args.n, seed=0)
    prm64 = ncorp.params_default(args.p, theta_min=args.theta, precision=ncorp.FP64,
                                 collision_mode=cmode, collision_f=2.0)
    prm32 = ncorp.params_default(args.p, theta_min=args.theta, precision=ncorp.FP32_BULK,
                                 collision_mode=cmode, collision_f=2.0)
    tuned = None
    if args.leaf_size == "auto":
        from paper_2310_20374_amd import autotune
        base = {k: torch.tensor(v, device=device) for k, v in d.items()}
        tuned = {}
        for name, prm, cands in (("fp32", prm32, LEAF_CANDIDATES_FP32),
                                 ("fp64", prm64, LEAF_CANDIDATES_FP64)):
            if name == "fp64" and args.fp32_only:
                continue
            tp, tab = autotune.tune_step(ncorp, prm, base, dt=args.dt, steps=3,
                                         leaf_sizes=cands, samples=min(args.samples, 2048),
                                         device=device)
            for k in ("leaf_size", "p2p_tile", "p2p_targets_max", "walk_waves"):
                setattr(prm, k, int(getattr(tp, k)))
            tuned[name] = {"leaf_size": int(prm.leaf_size),
                           "ms_per_step": {s: v["ms_per_step"] for s, v in tab["leaf_size"].items()},
                           "step_tuning": tab}
        del base
        print(f"# autotuned leaf sizes: {tuned}", file=sys.stderr, flush=True)
    else:
        prm32.leaf_size = prm64.leaf_size = int(args.leaf_size)
        if args.launch_shape:
            tile, waves = args.launch_shape.split(":")
            t, tmax = (int(v) for v in tile.split("x"))
            for prm in (prm32, prm64):
                prm.p2p_tile, prm.p2p_targets_max, prm.walk_waves = t, tmax, int(waves)
    thr = (prm64.ncs, prm64.ncc_pre, prm64.ncc_post)
    print(f"# bench: N={args.n} p={args.p} theta_min={args.theta} s={prm64.leaf_size} "
          f"steps={args.steps} warmup={args.warmup}", file=sys.stderr, flush=True)

    r32 = _run(ncorp, prm32, d, args.dt, args.steps, args.warmup, True, device)
    print(f"# fp32-bulk: {r32['wall_s'] * 1e3 / args.steps:.3f} ms/step", file=sys.stderr,
          flush=True)
    r64 = None
    if not args.fp32_only:
        r64 = _run(ncorp, prm64, d, args.dt, args.steps, args.warmup, True, device)
        print(f"# fp64: {r64['wall_s'] * 1e3 / args.steps:.3f} ms/step", file=sys.stderr,
              flush=True)

    thetas = [float(v) for v in args.thetas.split(",") if v.strip()]
    theta_runs = []
    for th in thetas:
        row = {"theta_min": th}
        for name, prm in (("fp32", prm32), ("fp64", prm64)):
            if name == "fp64" and args.fp32_only:
                continue
            p2 = ncorp.Params.from_buffer_copy(prm)
            p2.theta_min = th
            r = _run(ncorp, p2, d, args.dt, 10, 2, False, device)
            row[name] = {"ms_per_step": r["wall_s"] * 1e3 / 10, "acc": r["acc"],
                         "leaf_size": p2.leaf_size}
        theta_runs.append(row)
        print(f"# theta {th}: " + ", ".join(f"{k} {v['ms_per_step']:.3f} ms/step"
                                            for k, v in row.items() if k != "theta_min"),
              file=sys.stderr, flush=True)

    clustered = None
    if not args.no_clustered:
        clustered = _run_clustered(ncorp, args, device, prm32.leaf_size, cmode)
        print(f"# clustered: {clustered['ms_per_step']:.3f} ms/step, "
              f"{clustered['pairs_per_step']:.0f} pairs/step, "
              f"balance {clustered['load_balance']}", file=sys.stderr, flush=True)

    batched = None
    if not args.no_batched:
        batched = _run_batched(ncorp, args, device)
        print(f"# batched: {batched['ms_per_step']:.3f} ms/step (graph), "
              f"{batched['eager_ms_per_step']:.3f} eager, s={batched['leaf_size']}",
              file=sys.stderr, flush=True)

    mesh = mesh_acc = None
    if not args.no_mesh:
        mesh, mesh_acc = _run_mesh(ncorp, d, args, device)
        print(f"# mesh module: {mesh['ms_per_step']:.3f} ms/step, {mesh['mesh']}",
              file=sys.stderr, flush=True)

    methods = None
    if not args.no_method_comparison:
        methods = _gravity_method_comparison(ncorp, d, sorted({3, args.p}), 5, device,
                                             falcon_leaf=prm64.leaf_size)
        print("# gravity methods: " + ", ".join(
            f"{k} {v['ms_tree_and_gravity']:.3f} ms" for k, v in methods.items()),
            file=sys.stderr, flush=True)

    orc = None
    if not (args.no_errors and args.no_cpu_baseline):
        import oracle as orc
    err32 = err64 = None
    if not args.no_errors:
        err32 = _errors(orc, d, r32["acc"], args.samples)
        if r64 is not None:
            err64 = _errors(orc, d, r64["acc"], args.samples)
        print(f"# errors fp32 {err32} fp64 {err64}", file=sys.stderr, flush=True)
    for row in theta_runs:
        for name in ("fp32", "fp64"):
            if name in row:
                acc = row[name].pop("acc")
                if not args.no_errors:
                    row[name]["errors"] = _errors(orc, d, acc, args.samples)
    if clustered is not None:
        dcl = clustered.pop("_d")
        acc_cl = clustered.pop("_acc")
        got = clustered.pop("_pairs")
        if not args.no_errors:
            clustered["errors"] = _errors(orc, dcl, acc_cl, args.samples)
            want = orc.pairs_grid(dcl, args.dt)
            clustered["pair_check"] = {"dt": args.dt, "pairs": int(len(got)),
                                       "oracle_pairs": int(len(want)),
                                       "bit_exact": bool(np.array_equal(got, want))}
        del dcl, acc_cl, got
    if mesh is not None and not args.no_errors:
        mesh["errors"] = _errors(orc, d, mesh_acc, args.samples)
    if methods is not None:
        for v in methods.values():
            acc = v.pop("acc")
            if not args.no_errors:
                v["errors"] = _errors(orc, d, acc, args.samples)
        for p in sorted({3, args.p}):
            f, st = methods[f"falcon_p{p}"], methods[f"standard_tree_p{p}"]
            st["falcon_speedup"] = st["ms_tree_and_gravity"] / f["ms_tree_and_gravity"]
            st["falcon_speedup_collisions"] = st["ms_collision_search"] / f["ms_collision_search"]

    value = args.n * args.steps / r32["wall_s"]
    ph = r32["phases"]
    info = r32["info"]
    p2p_ms, p2p_launches = ph["p2p"]
    p2p_avg_s = p2p_ms / max(p2p_launches, 1) / 1e3
    flops = FLOPS_PER_INTERACTION * info["p2p_inter"]
    achieved = flops / p2p_avg_s / 1e12 if p2p_avg_s > 0 else 0.0
    roofline = {"bound": "alu",
                "kernel": "direct sums, FP32 VALU (k_p2p<float>, one "
                          "gravity evaluation)",
                "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": _p2p_traffic(args, prm32),
                "avg_launch_us": p2p_avg_s * 1e6, "launches": p2p_launches,
                "interactions_per_launch": info["p2p_inter"],
                "flops_per_interaction": FLOPS_PER_INTERACTION}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(orc, args.cpu_sample, args.p, args.theta, prm64.leaf_size, thr,
                            args.dt)
        cpu["cores"] = 1
        cpu["other_configs"] = _cpu_configs(orc, args.dt)

    phase_roof, step_frac = _phase_rooflines(ph, info, args.n, args.p, True)

    def phase_summary(r):
        if r is None or r["phases"] is None:
            return None
        return {k: round(v[0] / args.steps, 4) for k, v in r["phases"].items()}

    out = {
        "metric": "particle-steps/s (gravity+collision) at N=1M, FP32-bulk vs FP64, @RMS err",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "cold Keplerian disk of moonlets around a central mass (G=1, M=1): "
                        "lognormal masses summing to 0.01, a in [2.9,10], Rayleigh e 0.01 and "
                        "i 0.005; KDK steps with collision search + octree rebuild + falcON "
                        "gravity each step",
            "n": args.n, "p": args.p, "theta_min": args.theta, "theta_mode": "mass-dependent",
            "leaf_size": {"fp32": prm32.leaf_size, "fp64": prm64.leaf_size},
            "walk_thresholds": list(thr),
            "collision_thresholds": [prm64.ncs_col, prm64.ncc_pre_col, prm64.ncc_post_col],
            "dt": args.dt,
            "collisions": "resolved elastically (hard spheres, f = 2)" if args.collisions ==
                          "resolve" else "found and reported, not resolved",
            "precision": "fp32-bulk: direct sums and M2L in f32 (Kahan-summed "
                                        "tiles), positions/offsets/climbs/integrator in f64",
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "errors_fp32": err32,
        "fp64": None if r64 is None else {
            "value": args.n * args.steps / r64["wall_s"],
            "ms_per_step": r64["wall_s"] * 1e3 / args.steps, "errors": err64,
            "phases_ms_per_step": phase_summary(r64)},
        "phases_ms_per_step": phase_summary(r32),
        "phase_rooflines": phase_roof,
        "step_roofline_frac": step_frac,
        "tree": info,
        "collision_pairs_in_timed_steps": r32["pairs"],
        "batched": batched,
        "clustered": clustered,
        "gravity_methods": methods,
        "mesh_module": mesh,
        "leaf_size_autotune": tuned,
        "theta_sweep": theta_runs,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())

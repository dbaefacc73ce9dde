"""Shared helpers of the GPU tests (device arrays from the seeded generators)."""
import numpy as np


def dev_arrays(d, device="cuda:0"):
    import torch
    return {k: torch.tensor(np.ascontiguousarray(v), device=device) for k, v in d.items()}


def run_gravity(nc, d, prm, device="cuda:0", ctx=None):
    import torch
    n = len(d["x"])
    ctx = ctx or nc.Context(prm, n, pair_capacity=1 << 14, device=device)
    t = dev_arrays(d, device)
    a = [torch.empty(n, dtype=torch.float64, device=device) for _ in range(3)]
    ctx.build_tree(t["x"], t["y"], t["z"])
    ctx.gravity(t["m"], *a)
    torch.cuda.synchronize()
    ctx.check_status()
    return ctx, torch.stack(a, 1).cpu().numpy()


def run_collide(nc, d, prm, dt, cap=1 << 18, device="cuda:0", ctx=None):
    import torch
    n = len(d["x"])
    ctx = ctx or nc.Context(prm, n, pair_capacity=cap, device=device)
    t = dev_arrays(d, device)
    pairs = torch.zeros((cap, 2), dtype=torch.int64, device=device)
    npairs = torch.zeros(1, dtype=torch.int64, device=device)
    ctx.build_tree(t["x"], t["y"], t["z"])
    ctx.collide(t["vx"], t["vy"], t["vz"], t["R"], dt, pairs, npairs)
    torch.cuda.synchronize()
    ctx.check_status()
    k = int(npairs.item())
    return ctx, pairs[:k].cpu().numpy()


def rel_err(a, ref):
    e = np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return float(np.sqrt(np.mean(e * e))), float(e.max())

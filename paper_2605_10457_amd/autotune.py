"""Autotuner for the caster's tunables.

Searches the small/large split thresholds (gamma_T, chi_T) of the span
classification (Eq. sat_cond; the paper's default is (64, 64) and it sweeps
{32..128}^2), the per-channel work-item size, the bounds-pass block size and
the residency of the persistent kernels, by coordinate descent: one parameter
at a time over its candidate list, keeping the best, repeated until no change.
Each candidate is timed on the real workload with HIP events around a batched
cast (median of `reps`).  Every candidate gives bitwise-identical results
(the options only move work between classes), which `tune` verifies.

Results persist as JSON keyed by GPU architecture and workload signature.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import grca

SPACE = {
    "small_channels": [1, 2, 4, 8, 16, 32, 64],
    "small_rays": [8, 16, 32, 64, 128, 256],
    "row_chunk": [64, 128, 256, 512, 1024, 2048],
    "bounds_block": [128, 256, 512],
    "persist_waves_cu": [4, 8, 16, 24, 32],
    "group_cull": [0, 1],
    "isect_ticket": [512, 1024, 2048, 4096, 8192],
}
ORDER = ["group_cull", "small_channels", "small_rays", "row_chunk", "bounds_block",
         "persist_waves_cu", "isect_ticket"]
TUNING_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning")


def time_cast(torch, ctx, ids, dist, tri, reps: int = 5) -> float:
    st = torch.cuda.current_stream()
    ctx.cast(ids, dist, tri, stream=st)      # warm (and grow queues)
    ctx.synchronize(st)
    ms = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(st)
        ctx.cast(ids, dist, tri, stream=st)
        b.record(st)
        ctx.synchronize(st)
        ms.append(a.elapsed_time(b))
    return float(np.median(ms))


def tune(ctx, ids, n_rays: int, reps: int = 5, max_rounds: int = 2, log=None) -> dict:
    import torch
    dist = torch.empty(n_rays, dtype=torch.float32, device="cuda")
    tri = torch.empty(n_rays, dtype=torch.int32, device="cuda")
    best = {k: ctx.get_options()[k] for k in ORDER}
    ctx.set_options(**best)
    best_ms = time_cast(torch, ctx, ids, dist, tri, reps)
    ref_t = tri.clone()
    ref_d = dist.view(torch.int32).clone()
    history = [(dict(best), best_ms)]
    for rnd in range(max_rounds):
        changed = False
        for k in ORDER:
            for v in SPACE[k]:
                if v == best[k]:
                    continue
                cand = dict(best, **{k: v})
                ctx.set_options(**cand)
                ms = time_cast(torch, ctx, ids, dist, tri, reps)
                if not (torch.equal(tri, ref_t) and torch.equal(dist.view(torch.int32), ref_d)):
                    raise RuntimeError(f"options {cand} changed the result")
                history.append((cand, ms))
                if log:
                    log(f"tune round {rnd} {k}={v}: {ms:.3f} ms (best {best_ms:.3f})")
                if ms < best_ms * 0.99:
                    best, best_ms, changed = cand, ms, True
            ctx.set_options(**best)
        if not changed:
            break
    ctx.set_options(**best)
    return {"options": best, "ms": best_ms, "history": [[h, m] for h, m in history]}


def signature(workload) -> str:
    s = workload.sensors
    shape = "-".join(f"{len(x['elevation'])}x{x['rays_per_channel']}" for x in s)
    return f"{workload.name}_{workload.scene.num_triangles}_{shape}"


def save(result: dict, arch: str, name: str, sig: str) -> str:
    """Write the result for workload `name` (the file load() reads back)."""
    os.makedirs(TUNING_DIR, exist_ok=True)
    path = os.path.join(TUNING_DIR, f"{arch}_{name}.json")
    out = dict(result, arch=arch, signature=sig)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return path


def load(arch: str, name: str) -> dict | None:
    path = os.path.join(TUNING_DIR, f"{arch}_{name}.json")
    if os.path.exists(path):
        return json.load(open(path))
    return None


def main():
    import argparse
    import sys
    import time

    import torch

    from . import synth

    ap = argparse.ArgumentParser(description="tune the caster on a workload and save the result")
    ap.add_argument("--config", default="4",
                    help="1-4, or 'colocated' (config 4's scene seen by 2 rigs of 4 heads)")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--rounds", type=int, default=2)
    args = ap.parse_args()

    def log(m):
        print(f"[tune] {m}", file=sys.stderr, flush=True)

    t0 = time.time()
    wl = {"1": synth.config1, "2": synth.config2, "3": synth.config3,
          "4": lambda: synth.config4(scale=args.scale),
          "colocated": lambda: synth.config4_colocated(scale=args.scale)}[args.config]()
    log(f"{wl.name}: {wl.scene.num_triangles} tris in {time.time() - t0:.1f}s")
    ctx = grca.Context(0)
    ctx.set_options(item_capacity=96 << 20, large_capacity=8 << 20)
    ids = grca.load_workload(ctx, wl, frame=0)
    n = sum(len(s["elevation"]) * s["rays_per_channel"] for s in wl.sensors)
    res = tune(ctx, ids, n, reps=args.reps, max_rounds=args.rounds, log=log)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = save(res, arch, wl.name, signature(wl))
    log(f"best {res['options']} {res['ms']:.3f} ms -> {path}")
    print(json.dumps({"options": res["options"], "ms": res["ms"], "path": path}))
    ctx.close()


if __name__ == "__main__":
    main()

#!/usr/bin/env python
"""Frame benchmark of the emitter-centric caster on one MI355X.

Workload (default): 8 LiDARs of 128x4096 rays (4 x 360 deg, 4 x 180 deg facing
outward) on a 20 m ring over ~22M triangles of which ~9M are dynamic (20 rigid
vehicle proxies re-posed with a fresh random pose, per-axis scale and yaw
every frame, plus 10 sinusoidally deforming grids), range 0.05-1000 m.

A step is one frame: pose the dynamic geometry, then cast every ray of the 8
sensors (bounds + binning, large-class expansion, intersection, resolve).
  * batched: one hipGraph replay per frame (one 8-origin bounds pass, one
    persistent work queue for all sensors) -- this is `value`;
  * plain:   pose + one grca_cast per sensor, issued back to back, no graph.
Inputs are resident in HBM before the timed region; per-frame pose matrices
are generated beforehand and copied inside the frame (48 B per instance).

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rays/s + frame ms, 8×(128×4096) LiDARs on 22M tris; batched vs plain; p99"
HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed-FP32 instructions (the build disables them):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The published
# 157.3 TFLOP/s counts the packed (2-wide) FMA.
FP32_PEAK_TFLOPS = 78.6
FLOPS_PER_RTIC = 22               # ray test: 2 mul (direction) + 4 dot products x 5 flops
# Bounds pass, counting add/sub/mul/rsq/rcp/sqrt = 1, fma = 2 (compares,
# min/max, floor/ceil and selects not counted; work per sensor or per
# triangle alone, such as range thresholds and radii, not counted per pair):
# * bounding test of one (triangle, origin) pair: radius from the packed
#   cylinder 4, offset 3, local frame 15, |.|^2 5, distance 2, range 2,
#   angular margin 11 (the cylinder bound of an upright sensor; 6 for the
#   sphere's otherwise), sqrt 1, elevation atan2 19, channel-grid indices 6:
#   68 (63 for a sensor that is not upright);
# * the same test of a 128-triangle tile against one origin (its own packed
#   cylinder): 68 (63), plus, for a partial field of view, the wedge test (two
#   signed plane distances 3 + 3, margin 3): 9;
# * candidate span of one pair on the common path (no range or pole test,
#   azimuth offsets by the series bound): transform 54, |p|^2 15, sines 6,
#   edge bulge 27, margins 2, channel bins 4, atan2 of vertex 0 20, offsets of
#   vertices 1-2 28, full-turn test 1, azimuth margin 6, ray-index range 12.
FLOPS_PER_SPHERE = 68           # upright sensors
FLOPS_PER_SPHERE_TILTED = 63
FLOPS_PER_TILE_TEST = 68         # upright sensors (63 otherwise, as for triangles)
FLOPS_PER_WEDGE = 9
FLOPS_PER_SPAN = 175


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q)) if len(a) else float("nan")


def oracle_pose(scene, frame):
    """The oracle's own pose of the dynamic geometry (FP64, rounded to FP32)."""
    from oracle import oracle as O
    from paper_2605_10457_amd import synth
    v = scene.vertices.copy()
    if scene.rigid is not None:
        mats = scene.instance_matrices(frame)
        for i, (s, c) in enumerate(zip(scene.rigid.vertex_start, scene.rigid.vertex_count)):
            v[s:s + c] = O.pose_rigid(scene.vertices[s:s + c], mats[i])
    off = 0
    for g in scene.deform:
        s, c = g.vertex_start, g.vertex_count
        v[s:s + c] = O.pose_deform(scene.vertices[s:s + c], scene.deform_normals[off:off + c],
                                   scene.deform_phase[off:off + c], g.amplitude, g.omega,
                                   synth.deform_time(frame))
        off += c
    return v


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("grca_kernels.hip", "grca_device.hpp"):
        with open(os.path.join(ROOT, "paper_2605_10457_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_summary(paths) -> str:
    """Per-kernel mean of each counter over the dispatches of rocprofv3 CSVs."""
    import csv
    acc = {}
    for p in paths:
        with open(p) as fh:
            for row in csv.DictReader(fh):
                name = row.get("Kernel_Name", "?").split("(")[0].split("<")[0]
                key = (name, row.get("Counter_Name", "?"))
                acc.setdefault(key, []).append(float(row.get("Counter_Value", "nan")))
    lines = ["| kernel | counter | dispatches | mean per dispatch |", "|---|---|---|---|"]
    for (k, c), v in sorted(acc.items()):
        lines.append(f"| {k} | {c} | {len(v)} | {np.mean(v):.6g} |")
    return "\n".join(lines)


def load_traffic(kernel: str):
    """Measured HBM bytes per launch of `kernel` from profiles/, if the kernel
    sources are unchanged since the counters were taken; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic_config4.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = kv.get(f"{kernel}_bytes_per_launch")
    return float(v) if v else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--range-max", type=float, default=1000.0)
    ap.add_argument("--scale", type=float, default=1.0, help="scene size factor (1 = 22M tris)")
    ap.add_argument("--colocated", action="store_true",
                    help="the same scene seen by 2 rigs of 4 co-located 90-degree heads "
                         "(4.19M rays per frame) instead of the 8 ring sensors")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=16, help="oracle rays per sensor")
    ap.add_argument("--no-lossy", action="store_true",
                    help="skip the leg of the paper's lossy accelerations (timed casts and "
                         "their hit-distance match rate on the oracle sample)")
    ap.add_argument("--lossy-frames", type=int, default=1,
                    help="frames of the lossy leg's Hit%% floor (each adds an oracle sample of "
                         "--cpu-rays rays per sensor)")
    ap.add_argument("--serving-seconds", type=float, default=3.0,
                    help="seconds of Poisson arrivals of the serving leg (16 clients with "
                         "resident scenes; 0 to skip)")
    ap.add_argument("--ranges", default="10,50,100",
                    help="range_max values (m) of the range-culling sweep ('' to skip)")
    ap.add_argument("--range-steps", type=int, default=10)
    ap.add_argument("--origin-sweep", type=int, default=0,
                    help="also time frames of 1..N full-turn 128x4096 heads on the same scene, "
                         "distributed over the ring's origins vs sharing the first one")
    ap.add_argument("--tuning", default="auto",
                    help="JSON file of grca options; 'auto' (default) takes the autotuner's "
                         "saved result for this GPU and workload if there is one, 'none' the "
                         "library defaults")
    ap.add_argument("--opt", action="append", default=[], help="option override k=v")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device copy first (scale reference for PMC byte counters)")
    ap.add_argument("--pmc-summary", nargs="+", default=None,
                    help="summarise rocprofv3 counter_collection.csv files and exit")
    args = ap.parse_args()
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}); this "
              "build has no multi-GPU path. Sensors would shard across GPUs with a scene "
              "replica each (disjoint outputs, no exchange), or triangles would shard with "
              "one element-wise 64-bit MIN reduction of the packed keys.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_10457_amd import grca, synth

    t0 = time.time()
    if args.colocated:
        wl = synth.config4_colocated(range_max=args.range_max, scale=args.scale)
    else:
        wl = synth.config4(range_max=args.range_max, scale=args.scale)
    sc = wl.scene
    n_sens = len(wl.sensors)
    sizes = [len(s["elevation"]) * s["rays_per_channel"] for s in wl.sensors]
    n_rays = int(sum(sizes))
    log(f"workload: {sc.num_triangles} tris ({sc.n_dynamic_tris} dynamic), {n_rays} rays, "
        f"generated in {time.time() - t0:.1f}s")
    mats = [sc.instance_matrices(i) for i in range(args.warmup + args.steps + 1)]

    torch.cuda.init()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ctx = grca.Context(0)
    opts = {"item_capacity": 96 << 20, "large_capacity": 8 << 20}
    tuning = None
    if args.tuning == "auto":
        from paper_2605_10457_amd import autotune
        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        t = autotune.load(arch, wl.name)
        if t and t.get("signature") == autotune.signature(wl):
            opts.update(t["options"])
            tuning = f"{arch}_{wl.name}.json (autotuner)"
    elif args.tuning and args.tuning != "none" and os.path.exists(args.tuning):
        opts.update(json.load(open(args.tuning)).get("options", {}))
        tuning = args.tuning
    for kv in args.opt:
        k, v = kv.split("=")
        opts[k] = float(v) if k == "eps_area" else int(v)
    ctx.set_options(**opts)
    ids = grca.load_workload(ctx, wl, scene_id=0, frame=0, stream=stream)
    torch.cuda.synchronize()
    dist = torch.empty(n_rays, dtype=torch.float32, device=dev)
    tri = torch.empty(n_rays, dtype=torch.int32, device=dev)
    log(f"scene resident; options {ctx.get_options()}")
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del a, b

    # ---------------- batched: hipGraph frame
    frame = grca.grca_frame_create(ctx.h, 0, ids, dist, tri)
    for i in range(args.warmup):
        grca.grca_frame_launch(ctx.h, frame, mats[i], synth.deform_time(i), stream)
        grca.grca_frame_synchronize(ctx.h, frame, stream)
    torch.cuda.synchronize()
    log("batched warmup done")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    overflow_retimed = False
    for attempt in range(2):
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for k in range(args.steps):
            f = args.warmup + k
            ev[k][0].record(stream)
            grca.grca_frame_launch(ctx.h, frame, mats[f], synth.deform_time(f), stream)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall_batched = time.perf_counter() - t_start
        # every launch since the last synchronize is checked for a queue
        # overflow; a frame that dropped work would be a wrong, faster frame
        try:
            grca.grca_frame_synchronize(ctx.h, frame, stream)
            break
        except grca.GrcaError as e:
            if e.status != grca.GRCA_ERR_CAPACITY or attempt:
                raise
            log(f"timed frames overflowed their queues ({e}); timing again with grown queues")
            overflow_retimed = True
    stats = ctx.last_stats()
    # per-kernel device times: the same frames launched stage by stage with
    # HIP events between the stages, on the same stream
    stage_rows = []
    for k in range(args.steps):
        f = args.warmup + k
        stage_rows.append(grca.grca_frame_profile(ctx.h, frame, mats[f], synth.deform_time(f),
                                                  stream))
    b_ms = [a.elapsed_time(b) for a, b in ev]
    stage_ms = {k: float(np.mean([r[k] for r in stage_rows])) for k in grca.STAGES}
    log(f"batched: mean {np.mean(b_ms):.3f} ms p50 {pct(b_ms, 50):.3f} p99 {pct(b_ms, 99):.3f}; "
        f"stages {stage_ms}; stats {stats}")
    d_batched = dist.clone()
    t_batched = tri.clone()
    grca.grca_frame_destroy(frame)

    # ---------------- plain: pose + one cast per sensor, no graph
    p_ms = []
    if not args.no_plain:
        offs = np.cumsum([0] + sizes)
        for i in range(args.warmup):
            ctx.scene_pose(0, mats[i], synth.deform_time(i), stream)
            for s in range(n_sens):
                ctx.cast([ids[s]], dist[offs[s]:offs[s + 1]], tri[offs[s]:offs[s + 1]],
                         stream=stream)
            ctx.synchronize(stream)
        pev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        for k in range(args.steps):
            f = args.warmup + k
            pev[k][0].record(stream)
            ctx.scene_pose(0, mats[f], synth.deform_time(f), stream)
            for s in range(n_sens):
                ctx.cast([ids[s]], dist[offs[s]:offs[s + 1]], tri[offs[s]:offs[s + 1]],
                         stream=stream)
            pev[k][1].record(stream)
        torch.cuda.synchronize()
        ctx.synchronize(stream)
        p_ms = [a.elapsed_time(b) for a, b in pev]
        log(f"plain: mean {np.mean(p_ms):.3f} ms p50 {pct(p_ms, 50):.3f} p99 {pct(p_ms, 99):.3f}")
        same = bool(torch.equal(dist, d_batched) and torch.equal(tri, t_batched))
        log(f"plain == batched (last frame, bitwise): {same}")
    else:
        same = None

    mean_b = float(np.mean(b_ms))
    value = n_rays / (mean_b * 1e-3)

    # ---------------- range-culling sweep (batched frames at shorter range_max)
    sweep = {}
    for rng_s in [x for x in args.ranges.split(",") if x.strip()]:
        dmax = float(rng_s)
        for k, s in enumerate(wl.sensors):
            ctx.sensor_config(ids[k], dict(s, range_max=np.float32(dmax)), 0)
        fr2 = grca.grca_frame_create(ctx.h, 0, ids, dist, tri)
        for i in range(2):
            grca.grca_frame_launch(ctx.h, fr2, mats[i], synth.deform_time(i), stream)
            grca.grca_frame_synchronize(ctx.h, fr2, stream)
        sev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.range_steps)]
        for k in range(args.range_steps):
            f = args.warmup + k
            sev[k][0].record(stream)
            grca.grca_frame_launch(ctx.h, fr2, mats[f], synth.deform_time(f), stream)
            sev[k][1].record(stream)
        torch.cuda.synchronize()
        grca.grca_frame_synchronize(ctx.h, fr2, stream)
        s_ms = [a.elapsed_time(b) for a, b in sev]
        st2 = ctx.last_stats()
        sweep[f"{dmax:g}"] = {"mean_ms": float(np.mean(s_ms)), "p99_ms": pct(s_ms, 99),
                             "rays_per_s": n_rays / (float(np.mean(s_ms)) * 1e-3),
                             "rtic": st2["rtic"]}
        log(f"range_max {dmax:g} m: {sweep[f'{dmax:g}']}")
        grca.grca_frame_destroy(fr2)
    for k, s in enumerate(wl.sensors):
        ctx.sensor_config(ids[k], s, 0)

    # ---------------- roofline of the dominant kernel
    dom = max(("bounds", "expand", "isect"), key=lambda k: stage_ms[k])
    if dom == "isect":
        achieved = FLOPS_PER_RTIC * stats["rtic"] / (stage_ms["isect"] * 1e-3) / 1e12
        roof = {"kernel": "isect_kernel", "bound": "alu", "achieved": achieved,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                "traffic": load_traffic("isect_kernel"),
                "work": f"{FLOPS_PER_RTIC} FP32 flops x {stats['rtic']} RTIC per launch"}
    elif dom == "bounds":
        # VALU-bound: FP32 flops of the tests and spans the pass computed
        n_tiles = -(-int(sc.num_triangles) // 128) if opts.get("group_cull", 1) else 0
        tile_tests = n_tiles * n_sens
        wedge_tests = n_tiles * sum(1 for s in wl.sensors if float(s["fov"]) < 2 * np.pi - 1e-6)
        upright = all(abs(float(s["up"][0])) + abs(float(s["up"][1])) <= 1e-4
                      and float(s["up"][2]) > 0 for s in wl.sensors)
        per_tri = FLOPS_PER_SPHERE if upright else FLOPS_PER_SPHERE_TILTED
        per_tile = FLOPS_PER_TILE_TEST if upright else FLOPS_PER_SPHERE_TILTED
        flops = (per_tile * tile_tests + FLOPS_PER_WEDGE * wedge_tests +
                 per_tri * stats["sphere_tests"] +
                 FLOPS_PER_SPAN * stats["pairs_evaluated"])
        achieved = flops / (stage_ms["bounds"] * 1e-3) / 1e12
        roof = {"kernel": "bounds_kernel", "bound": "alu", "achieved": achieved,
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                "traffic": load_traffic("bounds_kernel"),
                "work": f"{per_tile} FP32 flops x {tile_tests} tile tests + "
                        f"{FLOPS_PER_WEDGE} x {wedge_tests} tile wedge tests + "
                        f"{per_tri} x {stats['sphere_tests']} triangle tests + "
                        f"{FLOPS_PER_SPAN} x {stats['pairs_evaluated']} (triangle, origin) spans "
                        f"per launch"}
    else:
        nbytes = 20 * stats["large_records"] + 20 * stats["row_items"]
        achieved = nbytes / (stage_ms[dom] * 1e-3) / 1e9
        roof = {"kernel": f"{dom}_kernel", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": load_traffic(f"{dom}_kernel"),
                "work": f"{nbytes} algorithmic bytes per launch"}
    rtic_s = stats["rtic"] / (stage_ms["isect"] * 1e-3)
    # the streaming passes against HBM, with their algorithmic bytes: pose
    # reads 12 B of rest position (+12 B normal and 4 B phase when deforming)
    # and writes the 16 B vertex record per dynamic vertex; init writes the
    # 8 B key of each ray; resolve reads it and writes 4 B distance + 4 B
    # triangle id
    n_rigid_v = int(np.sum(sc.rigid.vertex_count)) if sc.rigid is not None else 0
    n_def_v = int(sum(g.vertex_count for g in sc.deform))
    stream_bytes = {"pose": 28 * n_rigid_v + 44 * n_def_v, "init": 8 * n_rays,
                    "resolve": 16 * n_rays}
    streaming = {}
    for k, nb in stream_bytes.items():
        gbs = nb / (stage_ms[k] * 1e-3) / 1e9
        streaming[k] = {"bytes": int(nb), "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS}
    atomics = {"per_frame": int(stats["atomics"]),
               "per_s": stats["atomics"] / (stage_ms["isect"] * 1e-3),
               "per_rtic": stats["atomics"] / max(1, stats["rtic"])}

    # ---------------- CPU baseline: the oracle on a bounded sample
    cpu = None
    samples = {}  # frame -> [(rays, oracle result)] per sensor
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        from tests import parity
        v_or = oracle_pose(sc, args.warmup + args.steps - 1)
        rng = np.random.default_rng(7)
        tot_rays = 0
        t_cpu = 0.0
        threads = 0
        bad = 0
        counts = {}
        offs = np.cumsum([0] + sizes)
        d_np = d_batched.cpu().numpy()
        t_np = t_batched.cpu().numpy().view(np.uint32)
        for s_i, s in enumerate(wl.sensors):
            rays = np.sort(rng.choice(sizes[s_i], args.cpu_rays, replace=False)).astype(np.uint32)
            tc = time.perf_counter()
            orc = O.cast(s, v_or, sc.indices, rays=rays)
            t_cpu += time.perf_counter() - tc
            samples.setdefault(args.warmup + args.steps - 1, []).append((rays, orc))
            threads = orc["threads"]
            tot_rays += len(rays)
            sel = offs[s_i] + rays.astype(np.int64)
            rep = parity.check(s, v_or, sc.indices, orc, d_np[sel], t_np[sel])
            bad += rep["counts"]["clean_mismatch"] + rep["counts"]["flagged_unacceptable"]
            parity.merge(counts, rep["counts"])
        cpu = {"value": tot_rays / t_cpu, "unit": "rays/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{args.cpu_rays} seeded rays per sensor x {n_sens} sensors of the last "
                         f"timed frame, FP64 brute force over all {sc.num_triangles} triangles",
               "seconds": t_cpu, "extrapolated_frame_s": t_cpu * n_rays / tot_rays,
               "parity_on_sample": {"violations": int(bad), **counts}}
        log(f"cpu oracle: {tot_rays} rays in {t_cpu:.1f}s on {threads} threads; parity {counts} bad={bad}")

    origins = None
    if args.origin_sweep > 0:
        origins = origin_sweep(torch, ctx, stream, wl, mats, dist, tri, args)

    lossy = None
    if not args.no_lossy and samples:
        lossy = lossy_leg(torch, ctx, stream, wl, ids, sizes, mats, samples, args, dist, tri)

    out = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mean_b, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded generator; the paper's meshes are not available)",
        "config": {"workload": ("2 rigs of 4 co-located 90-deg heads 128x4096 at two ring "
                                "origins, " if args.colocated else
                                "8 LiDARs 128x4096 (4x360, 4x180 deg) on a 20 m ring, ") +
                               f"{sc.num_triangles} tris ({sc.n_dynamic_tris} dynamic: 20 rigid "
                               "vehicle proxies with full-instant pose + 10 deforming grids), "
                               f"range 0.05-{args.range_max:g} m; batched hipGraph frame",
                   "tuning": tuning,
                   "rays_per_frame": n_rays, "triangles": sc.num_triangles,
                   "dynamic_triangles": sc.n_dynamic_tris, "sensors": n_sens},
        "frame_ms": {"batched": {"mean": mean_b, "p50": pct(b_ms, 50), "p99": pct(b_ms, 99)},
                     "plain": ({"mean": float(np.mean(p_ms)), "p50": pct(p_ms, 50),
                                "p99": pct(p_ms, 99)} if p_ms else None)},
        "speedup_batched_vs_plain": (float(np.mean(p_ms)) / mean_b) if p_ms else None,
        "plain_equals_batched": same,
        "timed_frames_overflowed": overflow_retimed,
        "host_wall_ms_per_frame": wall_batched * 1e3 / args.steps,
        "stage_ms": stage_ms,
        "rtic_per_frame": stats["rtic"], "rtic_per_s": rtic_s,
        "isect_atomics": atomics,
        "streaming_hbm": streaming,
        "work": {k: stats[k] for k in ("pairs_tested", "sphere_tests", "pairs_evaluated", "rect_items",
                                       "large_records", "row_items")},
        "range_sweep": sweep,
        "roofline": roof,
        "cpu_baseline": cpu,
        "lossy": lossy,
    }
    if origins is not None:
        out["origin_sweep"] = origins
    ctx.close()
    out["serving"] = serving_leg(args.serving_seconds) if args.serving_seconds > 0 else None
    print(json.dumps(out), flush=True)


def lossy_leg(torch, ctx, stream, wl, ids, sizes, mats, samples, args, dist, tri) -> dict:
    """The paper's lossy accelerations (opt-in cast flags), each alone and all
    together, against the exact cast: median ms per batched cast of all
    sensors (grca_cast, device outputs, no graph) and the Hit% floor, the worst over
    the sampled frames of the share of sampled rays whose hit distance matches
    the FP64 oracle within 1 mm or that both miss (the paper's accuracy
    criterion), also over the rays the oracle sees hit."""
    from oracle import oracle as O
    from paper_2605_10457_amd import grca, synth
    from tests import parity
    modes = {"exact": 0, "area": grca.GRCA_LOSSY_AREA, "cspan": grca.GRCA_LOSSY_CSPAN,
             "rspan": grca.GRCA_LOSSY_RSPAN,
             "all": grca.GRCA_LOSSY_AREA | grca.GRCA_LOSSY_CSPAN | grca.GRCA_LOSSY_RSPAN}
    sc = wl.scene
    offs = np.cumsum([0] + sizes)
    frames = sorted(samples)
    rng = np.random.default_rng(11)
    while len(frames) < args.lossy_frames:  # more frames, each with its own oracle sample
        f = frames[-1] + 1
        v_or = oracle_pose(sc, f)
        samples[f] = []
        for s_i, s in enumerate(wl.sensors):
            rays = np.sort(rng.choice(sizes[s_i], args.cpu_rays, replace=False)).astype(np.uint32)
            samples[f].append((rays, O.cast(s, v_or, sc.indices, rays=rays)))
        frames.append(f)
    res = {m: {"ms": [], "rate": [], "rate_hits": [], "stats": None} for m in modes}
    for f in frames:
        ctx.scene_pose(0, sc.instance_matrices(f), synth.deform_time(f), stream)
        # the GPU idled through the oracle: bring its clocks back up first
        t_end = time.perf_counter() + 1.0
        while time.perf_counter() < t_end:
            for _ in range(20):
                ctx.cast(ids, dist, tri, stream=stream)
            ctx.synchronize(stream)
        for m, fl in modes.items():
            for _ in range(2):
                ctx.cast(ids, dist, tri, flags=fl, stream=stream)
            ctx.synchronize(stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(10)]
            for a, b in ev:
                a.record(stream)
                ctx.cast(ids, dist, tri, flags=fl, stream=stream)
                b.record(stream)
            ctx.synchronize(stream)
            res[m]["ms"] += [a.elapsed_time(b) for a, b in ev]
            res[m]["stats"] = ctx.last_stats()
            d = dist.cpu().numpy()
            match, match_h = [], []
            for s_i, (rays, orc) in enumerate(samples[f]):
                mk = parity.hit_match(orc, d[offs[s_i] + rays.astype(np.int64)])
                match.append(mk)
                match_h.append(mk[np.isfinite(orc["t"])])
            res[m]["rate"].append(float(np.mean(np.concatenate(match))))
            hh = np.concatenate(match_h)
            res[m]["rate_hits"].append(float(np.mean(hh)) if hh.size else 1.0)
    out = {}
    for m in modes:
        r = res[m]
        out[m] = {"ms": float(np.median(r["ms"])), "hit_floor": min(r["rate"]),
                  "hit_floor_on_hits": min(r["rate_hits"]),
                  "rtic": r["stats"]["rtic"], "rect_items": r["stats"]["rect_items"],
                  "large_records": r["stats"]["large_records"]}
        log(f"lossy {m}: {out[m]}")
    out["sample"] = (f"{args.cpu_rays} seeded rays per sensor x {len(wl.sensors)} sensors x "
                     f"{len(frames)} frame(s); match = hit distance within 1 mm of the FP64 "
                     f"oracle, or both miss")
    out["eps_area"] = ctx.get_options()["eps_area"]
    return out


def origin_sweep(torch, ctx, stream, wl, mats, dist, tri, args) -> dict:
    """Frames of 1..N full-turn 128x4096 heads on the workload's scene: one
    upright head at each of the first N ring origins (distributed), or N
    independently oriented heads sharing the first origin (co-located).  The
    paper's co-location experiment, on this scene; mean batched frame time
    and the pass's work counts."""
    from paper_2605_10457_amd import grca, synth
    origins = [s["origin"] for s in wl.sensors]
    kmax = min(args.origin_sweep, len(origins), dist.numel() // (128 * 4096))
    res = {"distributed": {}, "colocated": {}}
    for mode in res:
        for om in range(1, kmax + 1):
            sens = (synth.distributed_heads(origins[:om]) if mode == "distributed"
                    else synth.oriented_heads(origins[0], om))
            ids_s = list(range(300, 300 + om))
            for i, s in zip(ids_s, sens):
                ctx.sensor_config(i, s, 0)
            n = om * 128 * 4096
            fr = grca.grca_frame_create(ctx.h, 0, ids_s, dist[:n], tri[:n])
            for i in range(2):
                grca.grca_frame_launch(ctx.h, fr, mats[i], synth.deform_time(i), stream)
                grca.grca_frame_synchronize(ctx.h, fr, stream)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.range_steps)]
            for k in range(args.range_steps):
                f = args.warmup + k
                ev[k][0].record(stream)
                grca.grca_frame_launch(ctx.h, fr, mats[f], synth.deform_time(f), stream)
                ev[k][1].record(stream)
            torch.cuda.synchronize()
            grca.grca_frame_synchronize(ctx.h, fr, stream)
            st = ctx.last_stats()
            ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
            res[mode][str(om)] = {"ms": ms, "sphere_tests": st["sphere_tests"],
                                  "spans": st["pairs_evaluated"], "rtic": st["rtic"]}
            log(f"origin sweep {mode} x{om}: {res[mode][str(om)]}")
            grca.grca_frame_destroy(fr)
    return res


def serving_leg(seconds: float) -> dict:
    """Continuous-batching serving of 16 clients (their own resident scenes of
    0.5-4M triangles, 30-50% dynamic, 1-4 sensors each, Poisson arrivals at
    10-20 Hz per client): once in real time, once with the same arrivals
    compressed 50x so that the loop saturates.  Latency is host-clock time
    from arrival to outputs ready."""
    import torch
    from paper_2605_10457_amd import grca, serving
    t0 = time.time()
    ctx = grca.Context(0)
    ctx.set_options(item_capacity=64 << 20, large_capacity=4 << 20)
    clients = serving.make_clients(ctx, 16)
    for c in clients:                 # first-use allocations of every rig
        serving.solo(ctx, c, 0)
    torch.cuda.synchronize()
    res = {"clients": len(clients),
           "triangles": int(sum(c.workload.scene.num_triangles for c in clients)),
           "sensors": int(sum(len(c.sensor_ids) for c in clients)),
           "rays_per_round": int(sum(c.rays for c in clients)),
           "arrival_seconds": seconds}
    log(f"serving: {res} set up in {time.time() - t0:.1f}s")
    for name, ts in (("realtime", 1.0), ("saturated", 0.02)):
        reqs = serving.poisson_requests(clients, seconds, seed=11)
        srv = serving.Server(ctx, clients, slots=3)
        rep = srv.run(reqs, time_scale=ts)
        srv.close()
        rep["time_scale"] = ts
        res[name] = rep
        log(f"serving {name}: p50 {rep['latency_ms']['p50']:.2f} ms p99 "
            f"{rep['latency_ms']['p99']:.2f} ms, {rep['rays_per_s']:.3g} rays/s, "
            f"{rep['served']} served in {rep['batches']} batches (max {rep['max_batch']})")
    ctx.close()
    return res


if __name__ == "__main__":
    main()

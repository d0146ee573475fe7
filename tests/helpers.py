"""Helpers shared by the GPU tests: the oracle's pose of a workload's scene
and sampled parity of a batched cast against the oracle."""
from __future__ import annotations

import time

import numpy as np

from oracle import oracle as O
from paper_2605_10457_amd import synth
from tests import parity


def say(msg):
    print(f"[case] {msg}", flush=True)


def oracle_pose(scene, frame):
    """The scene's vertices at `frame`, posed by the oracle (FP64, rounded once)."""
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


def pick_rays(n, d_sensor, per_sensor, rng, hit_share=0.0):
    """`per_sensor` distinct ray ids of one sensor: a seeded uniform sample, of
    which a share `hit_share` is drawn among the rays the cast reports as hits
    (so that short-range casts, which miss almost everywhere, still check hits)."""
    k_hit = int(round(per_sensor * hit_share))
    hits = np.nonzero(np.isfinite(d_sensor))[0]
    k_hit = min(k_hit, hits.size)
    a = rng.choice(hits, k_hit, replace=False) if k_hit else np.empty(0, np.int64)
    rest = np.setdiff1d(np.arange(n), a)
    b = rng.choice(rest, min(per_sensor - k_hit, rest.size), replace=False)
    return np.sort(np.concatenate([a, b])).astype(np.uint32)


def sample_parity(sensors, v, f, d, t, per_sensor, seed, label, hit_share=0.0):
    """Oracle parity on `per_sensor` seeded rays of every sensor of a batched
    cast (outputs concatenated in sensor order); prints progress per sensor."""
    rng = np.random.default_rng(seed)
    off = 0
    tot = {}
    for k, s in enumerate(sensors):
        n = len(s["elevation"]) * s["rays_per_channel"]
        rays = pick_rays(n, d[off:off + n], per_sensor, rng, hit_share)
        t0 = time.perf_counter()
        orc = O.cast(s, v, f, rays=rays)
        sel = off + rays.astype(np.int64)
        rep = parity.check(s, v, f, orc, d[sel], t[sel])
        print(f"  {label} sensor {k}: {rays.size} rays, oracle {time.perf_counter() - t0:.1f} s, "
              f"{rep['counts']}", flush=True)
        parity.assert_parity(rep, f"{label} sensor {k}")
        parity.merge(tot, rep["counts"])
        off += n
    print(label, tot, flush=True)
    return tot

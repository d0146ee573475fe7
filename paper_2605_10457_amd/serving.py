"""Continuous-batching serving loop for LiDAR frame requests on one GPU.

Each client keeps its scene (static + dynamic geometry) and its sensor rig
resident in HBM for the whole run.  A frame request asks for one frame of one
client: pose the client's dynamic geometry at the request's simulation time,
then cast all of the client's sensors.

The scheduler owns K slots; a slot is a library workspace (ray keys, work
queues, counters) with its own HIP stream and output buffers.  Whenever a slot
is free it takes every admissible queued request -- requests of different
clients in one batch -- poses their scenes on the slot's stream and issues ONE
multi-scene cast over all their sensors.  Requests that arrive while other
batches are on the GPU join the next batch as soon as a slot and HBM budget
free up; batches on different slots overlap on the device.

Admission: a request's transient HBM is its rays x 16 B (key + outputs) plus
its share of the slot's work queues: 20 B per queued work item (16 B record +
4 B candidate start) and 16 B per large-class record, estimated per client
from a calibration cast of its rig (x 1.25 for pose-to-pose variation).  A
batch must fit its slot's ray capacity and queue capacity (so that no cast
overflows and regrows its queues mid-run) and the global transient budget.
A client has at most one request in flight (its scene is re-posed per
request).

Latency is measured on the host clock from arrival to outputs ready.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import grca, synth

BYTES_PER_RAY = 16    # 8 B key + 4 B distance + 4 B triangle id
BYTES_PER_ITEM = 20   # queued work item: 16 B record + 4 B first-candidate index
BYTES_PER_LARGE = 16  # large-class (triangle, origin) record
QUEUE_MARGIN = 1.25   # calibration estimate -> admission estimate


@dataclasses.dataclass
class Client:
    cid: int
    workload: synth.Workload
    scene_id: int
    sensor_ids: list
    rays: int
    rate_hz: float
    items: int = 0   # queued work items of one request (calibration estimate)
    large: int = 0   # large-class records of one request (calibration estimate)

    def transient_bytes(self) -> int:
        return (self.rays * BYTES_PER_RAY + self.items * BYTES_PER_ITEM
                + self.large * BYTES_PER_LARGE)


@dataclasses.dataclass(order=True)
class Request:
    arrival: float
    rid: int = dataclasses.field(compare=False)
    cid: int = dataclasses.field(compare=False)
    frame: int = dataclasses.field(compare=False)
    done: float = dataclasses.field(default=math.nan, compare=False)
    slot: int = dataclasses.field(default=-1, compare=False)
    batch: int = dataclasses.field(default=-1, compare=False)
    offset: int = dataclasses.field(default=0, compare=False)


def plan_batch(queue, need: dict, busy: set, slot_max_rays: int, slot_max_items: int,
               budget_bytes: int, in_use_bytes: int):
    """Admission for one free slot: oldest requests first, at most one per
    client, skipping clients with a request in flight; a request joins the
    batch while the batch fits the slot's ray and queue capacities and the
    transient HBM budget.  `need[cid]` = (rays, queue items, transient bytes)
    of one request of client cid.  Requests that can never fit (larger than a
    slot or the whole budget) are rejected.  Returns (batch, still_queued,
    rejected)."""
    batch, keep, rejected = [], [], []
    taken = set()
    rays = items = nbytes = 0
    for r in sorted(queue):
        n_r, n_i, n_b = need[r.cid]
        if n_r > slot_max_rays or n_i > slot_max_items or n_b > budget_bytes:
            rejected.append(r)
            continue
        if r.cid in busy or r.cid in taken:
            keep.append(r)
            continue
        if (rays + n_r > slot_max_rays or items + n_i > slot_max_items
                or in_use_bytes + nbytes + n_b > budget_bytes):
            keep.append(r)
            continue
        batch.append(r)
        taken.add(r.cid)
        rays += n_r
        items += n_i
        nbytes += n_b
    return batch, keep, rejected


class Slot:
    def __init__(self, torch, ctx, idx, max_rays, item_cap):
        self.idx = idx
        self.ws, self.bytes = grca.grca_workspace_create(ctx.h, max_rays, item_cap)
        self.stream = torch.cuda.Stream()
        self.dist = torch.empty(max_rays, dtype=torch.float32, device="cuda")
        self.tri = torch.empty(max_rays, dtype=torch.int32, device="cuda")
        self.max_rays = max_rays
        self.max_items = item_cap
        self.event = None
        self.reqs: list[Request] = []
        self.rays = 0
        self.nbytes = 0


class Server:
    def __init__(self, ctx: grca.Context, clients: list[Client], slots: int = 3,
                 max_rays_per_slot: int = 16 << 20, item_cap: int = 64 << 20,
                 transient_budget_bytes: int = 32 << 30, keep_outputs: set | None = None):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.clients = {c.cid: c for c in clients}
        self.slots = [Slot(torch, ctx, i, max_rays_per_slot, item_cap) for i in range(slots)]
        self.budget = transient_budget_bytes
        self.in_use = 0
        self.busy_clients: set = set()
        self.keep = keep_outputs or set()
        self.outputs: dict = {}
        self.batches = 0
        self.admitted = 0
        self.rejected = 0
        self.max_batch = 0
        self.overflowed = 0
        self.need = {c.cid: (c.rays, int(math.ceil(c.items * QUEUE_MARGIN)),
                             int(math.ceil(c.transient_bytes() * QUEUE_MARGIN)))
                     for c in clients}

    # -------------------------------------------------------------- batching
    def _launch(self, slot: Slot, reqs: list[Request], now: float):
        ids, off, nbytes = [], 0, 0
        for r in reqs:
            c = self.clients[r.cid]
            sc = c.workload.scene
            mats = sc.instance_matrices(r.frame) if sc.rigid is not None else None
            if sc.rigid is not None or sc.deform:
                self.ctx.scene_pose(c.scene_id, mats, synth.deform_time(r.frame), slot.stream)
            r.offset = off
            r.slot = slot.idx
            r.batch = self.batches
            ids.extend(c.sensor_ids)
            off += c.rays
            nbytes += self.need[r.cid][2]
            self.busy_clients.add(r.cid)
        grca.grca_cast_ws(self.ctx.h, slot.ws, ids, slot.dist, slot.tri, slot.stream)
        ev = self.torch.cuda.Event()
        ev.record(slot.stream)
        slot.event = ev
        slot.reqs = reqs
        slot.rays = off
        slot.nbytes = nbytes
        self.in_use += nbytes
        self.batches += 1
        self.max_batch = max(self.max_batch, len(reqs))

    def _complete(self, slot: Slot, now: float):
        grca.grca_workspace_synchronize(self.ctx.h, slot.ws, slot.stream)
        self.overflowed += grca.grca_workspace_stats(self.ctx.h, slot.ws)["overflowed"]
        for r in slot.reqs:
            r.done = now
            self.busy_clients.discard(r.cid)
            if r.rid in self.keep:
                c = self.clients[r.cid]
                d = slot.dist[r.offset:r.offset + c.rays].cpu().numpy().copy()
                t = slot.tri[r.offset:r.offset + c.rays].cpu().numpy().view(np.uint32).copy()
                self.outputs[r.rid] = (d, t)
        self.in_use -= slot.nbytes
        slot.event = None
        slot.reqs = []
        slot.rays = 0
        slot.nbytes = 0

    def _admit(self, queue: list, slot: Slot) -> list:
        batch, keep, rejected = plan_batch(queue, self.need, self.busy_clients, slot.max_rays,
                                           slot.max_items, self.budget, self.in_use)
        queue[:] = keep
        self.rejected += len(rejected)
        self.admitted += len(batch)
        return batch

    # -------------------------------------------------------------- run loop
    def run(self, requests: list[Request], time_scale: float = 1.0, log=None) -> dict:
        """Serve `requests` (arrival times in seconds from start, real clock)."""
        pending = list(sorted(requests))
        queue: list[Request] = []
        t0 = time.perf_counter()
        nxt = 0
        total = len(pending)
        completed = 0
        last_log = t0
        while completed + self.rejected < total:
            now = time.perf_counter() - t0
            while nxt < total and pending[nxt].arrival * time_scale <= now:
                queue.append(pending[nxt])
                nxt += 1
            for s in self.slots:
                if s.event is not None and s.event.query():
                    completed += len(s.reqs)
                    self._complete(s, time.perf_counter() - t0)
            for s in self.slots:
                if s.event is None and queue:
                    b = self._admit(queue, s)
                    if b:
                        self._launch(s, b, now)
            if log and time.perf_counter() - last_log > 5.0:
                last_log = time.perf_counter()
                log(f"served {completed}/{total} queued {len(queue)} batches {self.batches}")
            if all(s.event is None for s in self.slots) and not queue and nxt < total:
                wait = pending[nxt].arrival * time_scale - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.002))
            else:
                time.sleep(0.0002)
        wall = time.perf_counter() - t0
        lat = np.array([(r.done - r.arrival * time_scale) * 1e3 for r in pending
                        if not math.isnan(r.done)])
        rays = sum(self.clients[r.cid].rays for r in pending if not math.isnan(r.done))
        return {
            "requests": total, "served": int(lat.size), "rejected": self.rejected,
            "batches": self.batches, "max_batch": self.max_batch,
            "latency_ms": {"p50": float(np.percentile(lat, 50)) if lat.size else None,
                           "p99": float(np.percentile(lat, 99)) if lat.size else None,
                           "mean": float(lat.mean()) if lat.size else None},
            "rays_per_s": rays / wall, "wall_s": wall,
            "slot_bytes": [s.bytes for s in self.slots],
            "casts_overflowed": self.overflowed,
        }

    def close(self):
        for s in self.slots:
            if s.event is not None:
                s.event.synchronize()
            grca.grca_workspace_destroy(s.ws)
        self.slots = []


def make_clients(ctx: grca.Context, n_clients: int = 16, tri_scale: float = 1.0,
                 seed_extra: int = 0, log=None) -> list[Client]:
    """Build and upload the clients' resident scenes and rigs (config 5 recipe)."""
    clients = []
    next_sensor = 0
    for c in range(n_clients):
        wl = synth.client_workload(c, seed_extra=seed_extra, tri_scale=tri_scale)
        ids = grca.load_workload(ctx, wl, scene_id=1000 + c, first_sensor_id=next_sensor, frame=0)
        next_sensor += len(ids)
        rays = sum(len(s["elevation"]) * s["rays_per_channel"] for s in wl.sensors)
        rng = np.random.default_rng([synth.BASE_SEED + 5 + seed_extra, c, 99])
        cl = Client(c, wl, 1000 + c, ids, rays, float(rng.uniform(10, 20)))
        # calibration cast: the rig's queue demand at the resident pose
        ctx.cast_host(ids, rays)
        st = ctx.last_stats()
        cl.items = int(st["rect_items"] + st["row_items"])
        cl.large = int(st["large_records"])
        clients.append(cl)
        if log:
            log(f"client {c}: {wl.scene.num_triangles} tris ({wl.scene.n_dynamic_tris} dyn), "
                f"{len(ids)} sensors, {rays} rays, {cl.items} queue items, "
                f"{cl.rate_hz:.1f} Hz")
    return clients


def poisson_requests(clients: list[Client], duration_s: float, seed: int = 0) -> list[Request]:
    rng = np.random.default_rng(seed)
    reqs = []
    rid = 0
    for c in clients:
        t = 0.0
        frame = 0
        while True:
            t += rng.exponential(1.0 / c.rate_hz)
            if t >= duration_s:
                break
            reqs.append(Request(t, rid, c.cid, frame))
            rid += 1
            frame += 1
    return reqs


def solo(ctx: grca.Context, client: Client, frame: int):
    """The request's result when cast alone (for the batched == alone check)."""
    sc = client.workload.scene
    mats = sc.instance_matrices(frame) if sc.rigid is not None else None
    if sc.rigid is not None or sc.deform:
        ctx.scene_pose(client.scene_id, mats, synth.deform_time(frame))
    return ctx.cast_host(client.sensor_ids, client.rays)


def main(argv=None):
    """Serving benchmark of the config 5 recipe: `n` clients with resident
    scenes and rigs, Poisson frame arrivals at 10-20 Hz per client.  Runs the
    arrivals once in real time and once compressed in time (offered load far
    above what the GPU can serve, so batches fill and the loop saturates), and
    prints one JSON line with p50/p99 latency and aggregate rays/s of each."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(prog="python -m paper_2605_10457_amd.serving")
    ap.add_argument("--clients", type=int, default=16)
    ap.add_argument("--duration", type=float, default=10.0, help="seconds of arrivals")
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--saturate-scale", type=float, default=0.02,
                    help="time compression of the saturated run (0 to skip)")
    ap.add_argument("--tri-scale", type=float, default=1.0)
    args = ap.parse_args(argv)

    def log(m):
        print(f"[serving] {m}", file=sys.stderr, flush=True)

    import torch
    torch.cuda.init()
    ctx = grca.Context(0)
    ctx.set_options(item_capacity=64 << 20, large_capacity=4 << 20)
    clients = make_clients(ctx, args.clients, tri_scale=args.tri_scale, log=log)
    torch.cuda.synchronize()
    out = {"clients": len(clients),
           "triangles": int(sum(c.workload.scene.num_triangles for c in clients)),
           "sensors": int(sum(len(c.sensor_ids) for c in clients)),
           "rays_per_round": int(sum(c.rays for c in clients))}
    # warm every client once (first-use allocations), then serve
    for c in clients:
        solo(ctx, c, 0)
    runs = [("realtime", 1.0)]
    if args.saturate_scale > 0:
        runs.append(("saturated", args.saturate_scale))
    for name, ts in runs:
        reqs = poisson_requests(clients, args.duration, seed=11)
        srv = Server(ctx, clients, slots=args.slots)
        log(f"{name}: {len(reqs)} requests over {args.duration * ts:.2f} s")
        rep = srv.run(reqs, time_scale=ts, log=log)
        srv.close()
        rep["time_scale"] = ts
        out[name] = rep
        log(f"{name}: {rep}")
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()

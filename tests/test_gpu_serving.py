"""GPU test of the continuous-batching serving loop: requests from several
clients are batched into shared multi-scene casts on overlapping slots, and
every sampled request's result equals the same request cast alone."""
import numpy as np
import pytest

from paper_2605_10457_amd import grca, serving
from tests import parity

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_alone():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] serving: 6 small clients, 2 s of Poisson arrivals, 3 slots", flush=True)
    ctx = grca.Context(0)
    try:
        clients = serving.make_clients(ctx, n_clients=6, tri_scale=0.02)
        reqs = serving.poisson_requests(clients, duration_s=2.0, seed=1)
        keep = {r.rid for r in reqs[::7]}
        srv = serving.Server(ctx, clients, slots=3, max_rays_per_slot=6 << 20,
                             item_cap=16 << 20, transient_budget_bytes=2 << 30, keep_outputs=keep)
        # arrivals compressed 20x so that requests queue up behind batches in flight
        rep = srv.run(reqs, time_scale=0.05)
        print("serving", rep, flush=True)
        assert rep["served"] == len(reqs) and rep["rejected"] == 0
        assert rep["max_batch"] >= 2, "requests from different clients never shared a batch"
        byid = {r.rid: r for r in reqs}
        for rid, (d, t) in srv.outputs.items():
            r = byid[rid]
            d1, t1 = serving.solo(ctx, srv.clients[r.cid], r.frame)
            assert np.array_equal(t, t1), f"request {rid}: mix != alone"
            assert np.array_equal(d.view(np.uint32), d1.view(np.uint32))
        srv.close()
    finally:
        ctx.close()


def test_serving_tight_budget_queues_instead_of_failing():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("[case] serving with a transient budget below two requests", flush=True)
    ctx = grca.Context(0)
    try:
        clients = serving.make_clients(ctx, n_clients=3, tri_scale=0.01, seed_extra=3)
        biggest = max(c.rays for c in clients)
        reqs = serving.poisson_requests(clients, duration_s=1.0, seed=2)
        srv = serving.Server(ctx, clients, slots=2, max_rays_per_slot=biggest,
                             item_cap=8 << 20, transient_budget_bytes=1 << 40)
        # a budget of the largest request's transient bytes (keys, outputs and
        # its share of the work queues): requests are admitted one at a time
        needs = sorted(n[2] for n in srv.need.values())
        assert all(c.items > 0 for c in clients)
        srv.budget = needs[-1]
        rep = srv.run(reqs)
        print("tight", rep, flush=True)
        assert rep["served"] == len(reqs) and rep["rejected"] == 0
        if needs[0] + needs[1] > needs[-1]:
            assert rep["max_batch"] == 1
        assert rep["casts_overflowed"] == 0
        srv.close()
    finally:
        ctx.close()


def test_serving_oracle_sample_full_scale():
    """16 clients with their full-size scenes (0.5-4M triangles each): a
    seeded 5% of the served requests (at most 12) is checked against the
    oracle on 64 rays per sensor, at the request's own frame, and re-cast
    alone for bitwise equality."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from tests import helpers
    print("[case] serving: 16 full-size clients, 1.5 s of Poisson arrivals, 3 slots, "
          "oracle on a 5% sample", flush=True)
    ctx = grca.Context(0)
    try:
        ctx.set_options(item_capacity=64 << 20, large_capacity=4 << 20)
        clients = serving.make_clients(ctx, n_clients=16)
        reqs = serving.poisson_requests(clients, duration_s=1.5, seed=5)
        rng = np.random.default_rng(55)
        n_pick = min(12, max(1, int(round(0.05 * len(reqs)))))
        keep = {reqs[i].rid for i in rng.choice(len(reqs), n_pick, replace=False)}
        srv = serving.Server(ctx, clients, slots=3, keep_outputs=keep)
        rep = srv.run(reqs)
        print("serving", rep, flush=True)
        assert rep["served"] == len(reqs) and rep["rejected"] == 0
        byid = {r.rid: r for r in reqs}
        tot = {}
        for rid, (d, t) in sorted(srv.outputs.items()):
            r = byid[rid]
            c = srv.clients[r.cid]
            sc = c.workload.scene
            v_or = helpers.oracle_pose(sc, r.frame)
            got = helpers.sample_parity(c.workload.sensors, v_or, sc.indices, d, t, 64,
                                        1000 + rid, f"request {rid} (client {r.cid}, "
                                        f"frame {r.frame}, {sc.num_triangles} tris)")
            parity.merge(tot, got)
            d1, t1 = serving.solo(ctx, c, r.frame)
            assert np.array_equal(t, t1), f"request {rid}: mix != alone"
            assert np.array_equal(d.view(np.uint32), d1.view(np.uint32))
        assert len(srv.outputs) == n_pick
        print("serving oracle sample", tot, flush=True)
        srv.close()
    finally:
        ctx.close()

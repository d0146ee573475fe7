"""GPU test of the continuous-batching serving loop: requests from several
clients are batched into shared multi-scene casts on overlapping slots, and
every sampled request's result equals the same request cast alone."""
import numpy as np
import pytest

from paper_2605_10457_amd import grca, serving

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
                             item_cap=8 << 20, transient_budget_bytes=biggest * 16)
        rep = srv.run(reqs)
        print("tight", rep, flush=True)
        assert rep["served"] == len(reqs)
        assert rep["max_batch"] == 1
        srv.close()
    finally:
        ctx.close()

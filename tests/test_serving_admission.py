"""CPU tests of the serving admission policy (no GPU needed)."""
from paper_2605_10457_amd.serving import (BYTES_PER_ITEM, BYTES_PER_LARGE, BYTES_PER_RAY,
                                          Client, Request, plan_batch)


def _q(*specs):
    return [Request(t, i, c, 0) for i, (t, c) in enumerate(specs)]


def _need(rays, items=None):
    """need[cid] = (rays, queue items, transient bytes) with no queue demand unless given."""
    items = items or {}
    return {c: (r, items.get(c, 0), r * BYTES_PER_RAY + items.get(c, 0) * BYTES_PER_ITEM)
            for c, r in rays.items()}


BIG = 1 << 40


def test_batches_different_clients_oldest_first():
    q = _q((0.3, 1), (0.1, 0), (0.2, 2))
    batch, keep, rej = plan_batch(q, _need({0: 100, 1: 100, 2: 100}), set(), 1000, BIG, BIG, 0)
    assert [r.cid for r in batch] == [0, 2, 1] and not keep and not rej


def test_one_request_per_client_and_busy_clients_wait():
    q = _q((0.1, 0), (0.2, 0), (0.3, 1), (0.4, 2))
    batch, keep, rej = plan_batch(q, _need({0: 10, 1: 10, 2: 10}), {2}, 1000, BIG, BIG, 0)
    assert [r.cid for r in batch] == [0, 1]
    assert sorted(r.cid for r in keep) == [0, 2] and not rej


def test_slot_capacity_and_budget_queue_instead_of_failing():
    q = _q((0.1, 0), (0.2, 1), (0.3, 2))
    need = _need({0: 600, 1: 600, 2: 300})
    batch, keep, rej = plan_batch(q, need, set(), 1000, BIG, BIG, 0)
    assert [r.cid for r in batch] == [0, 2] and [r.cid for r in keep] == [1]
    # budget below two requests: one at a time
    batch, keep, rej = plan_batch(q, need, set(), 10_000, BIG, 700 * BYTES_PER_RAY, 0)
    assert [r.cid for r in batch] == [0] and len(keep) == 2 and not rej
    # budget already used by batches in flight: nothing fits now, all wait
    batch, keep, rej = plan_batch(q, need, set(), 10_000, BIG, 700 * BYTES_PER_RAY,
                                  600 * BYTES_PER_RAY)
    assert not batch and len(keep) == 3


def test_queue_demand_counts_against_slot_and_budget():
    q = _q((0.1, 0), (0.2, 1), (0.3, 2))
    # few rays but large queue demand: the slot's queue capacity limits the batch
    need = _need({0: 10, 1: 10, 2: 10}, {0: 5000, 1: 5000, 2: 100})
    batch, keep, rej = plan_batch(q, need, set(), 1000, 6000, BIG, 0)
    assert [r.cid for r in batch] == [0, 2] and [r.cid for r in keep] == [1]
    # and the budget counts queue bytes, not only the 16 B per ray
    budget = 10 * BYTES_PER_RAY * 3 + 6000 * BYTES_PER_ITEM
    batch, keep, rej = plan_batch(q, need, set(), 1000, BIG, budget, 0)
    assert [r.cid for r in batch] == [0, 2]
    # a request whose queue demand alone exceeds a slot is rejected
    batch, keep, rej = plan_batch(q, need, set(), 1000, 4000, BIG, 0)
    assert [r.cid for r in rej] == [0, 1] and [r.cid for r in batch] == [2]


def test_requests_that_can_never_fit_are_rejected():
    q = _q((0.1, 0), (0.2, 1))
    batch, keep, rej = plan_batch(q, _need({0: 5000, 1: 10}), set(), 1000, BIG, BIG, 0)
    assert [r.cid for r in rej] == [0] and [r.cid for r in batch] == [1]


def test_client_transient_bytes():
    c = Client(0, None, 0, [0], rays=1000, rate_hz=10.0, items=50, large=3)
    assert c.transient_bytes() == 1000 * BYTES_PER_RAY + 50 * BYTES_PER_ITEM + 3 * BYTES_PER_LARGE

"""CPU tests of the serving admission policy (no GPU needed)."""
from paper_2605_10457_amd.serving import BYTES_PER_RAY, Request, plan_batch


def _q(*specs):
    return [Request(t, i, c, 0) for i, (t, c) in enumerate(specs)]


def test_batches_different_clients_oldest_first():
    q = _q((0.3, 1), (0.1, 0), (0.2, 2))
    batch, keep, rej = plan_batch(q, {0: 100, 1: 100, 2: 100}, set(), 1000, 1 << 30, 0)
    assert [r.cid for r in batch] == [0, 2, 1] and not keep and not rej


def test_one_request_per_client_and_busy_clients_wait():
    q = _q((0.1, 0), (0.2, 0), (0.3, 1), (0.4, 2))
    batch, keep, rej = plan_batch(q, {0: 10, 1: 10, 2: 10}, {2}, 1000, 1 << 30, 0)
    assert [r.cid for r in batch] == [0, 1]
    assert sorted(r.cid for r in keep) == [0, 2] and not rej


def test_slot_capacity_and_budget_queue_instead_of_failing():
    q = _q((0.1, 0), (0.2, 1), (0.3, 2))
    rays = {0: 600, 1: 600, 2: 300}
    batch, keep, rej = plan_batch(q, rays, set(), 1000, 1 << 30, 0)
    assert [r.cid for r in batch] == [0, 2] and [r.cid for r in keep] == [1]
    # budget below two requests: one at a time
    batch, keep, rej = plan_batch(q, rays, set(), 10_000, 700 * BYTES_PER_RAY, 0)
    assert [r.cid for r in batch] == [0] and len(keep) == 2 and not rej
    # budget already used by batches in flight: nothing fits now, all wait
    batch, keep, rej = plan_batch(q, rays, set(), 10_000, 700 * BYTES_PER_RAY,
                                  600 * BYTES_PER_RAY)
    assert not batch and len(keep) == 3


def test_requests_that_can_never_fit_are_rejected():
    q = _q((0.1, 0), (0.2, 1))
    batch, keep, rej = plan_batch(q, {0: 5000, 1: 10}, set(), 1000, 1 << 30, 0)
    assert [r.cid for r in rej] == [0] and [r.cid for r in batch] == [1]

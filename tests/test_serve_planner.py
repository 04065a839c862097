"""Admission policy of the server (no GPU): FIFO batching into bucketed
slots under an HBM budget."""

import numpy as np
import pytest

class _Req:
    def __init__(self, rid, n, grad=False):
        self.rid, self.n, self.grad, self.error = rid, n, grad, None

    @property
    def kind(self):
        return "grad" if self.grad else "fwd"


@pytest.fixture(scope="module")
def S():
    # importing the server touches no GPU (the binding only loads the library)
    import paper_2112_06830_amd.serve as S
    return S


def test_fifo_batches_fit_largest_bucket(S):
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 20}, budget_bytes=10**9,
                           max_inflight_per_kind=2)
    for i, n in enumerate([50, 60, 200, 90, 30]):
        assert p.enqueue(_Req(i, n))
    take, bucket = p.next_batch("fwd")
    assert [r.rid for r in take] == [0, 1, 2, 3] and bucket == 400
    take2, bucket2 = p.next_batch("fwd")
    assert [r.rid for r in take2] == [4] and bucket2 == 100
    assert p.next_batch("fwd") is None


def test_one_batch_in_flight_per_kind_absorbs_arrivals(S):
    # while a batch runs, arrivals queue and leave together as the next batch
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 20}, budget_bytes=10**9)
    p.enqueue(_Req(0, 50))
    take, bucket = p.next_batch("fwd")
    assert [r.rid for r in take] == [0] and bucket == 100
    for i in range(1, 4):
        p.enqueue(_Req(i, 60))
    assert p.next_batch("fwd") is None            # the kind's batch is still running
    p.enqueue(_Req(9, 10, grad=True))
    assert [r.rid for r in p.next_batch("grad")[0]] == [9]   # other kind unaffected
    p.release("fwd", 100)
    take, bucket = p.next_batch("fwd")
    assert [r.rid for r in take] == [1, 2, 3] and bucket == 400


def test_smallest_fitting_bucket_preferred_over_idle_larger(S):
    # an idle 400-slot exists, but a new 100-slot fits the budget: take it
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 10}, budget_bytes=10**9)
    p.enqueue(_Req(0, 350))
    p.next_batch("fwd")
    p.release("fwd", 400)
    p.enqueue(_Req(1, 50))
    take, b = p.next_batch("fwd")
    assert b == 100 and p.reserved == 5000 and not p.evicted


def test_budget_limits_slots_and_release_reuses(S):
    # one 400-slot of fwd costs 4000 bytes; the budget allows exactly one
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 20}, budget_bytes=4500, slots_per_bucket=2,
                           max_inflight_per_kind=2)
    for i in range(3):
        p.enqueue(_Req(i, 300))
    first = p.next_batch("fwd")
    assert first is not None and first[1] == 400
    assert p.next_batch("fwd") is None            # second slot would exceed the budget
    assert p.reserved <= p.budget
    p.release("fwd", 400)
    second = p.next_batch("fwd")                  # reuses the released slot
    assert second is not None and [r.rid for r in second[0]] == [1]
    assert p.reserved == 4000


def test_oversize_request_rejected(S):
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 20}, budget_bytes=10**9)
    r = _Req(0, 401)
    assert not p.enqueue(r) and "exceeds" in r.error
    p2 = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 20}, budget_bytes=3000)
    r2 = _Req(1, 350)     # needs a 400-slot = 4000 bytes > budget
    assert not p2.enqueue(r2)


def test_kinds_queue_separately(S):
    p = S.AdmissionPlanner([100], {"fwd": 1, "grad": 1}, budget_bytes=10**9)
    p.enqueue(_Req(0, 10, grad=True))
    p.enqueue(_Req(1, 10, grad=False))
    assert [r.rid for r in p.next_batch("grad")[0]] == [0]
    assert [r.rid for r in p.next_batch("fwd")[0]] == [1]


def test_trace_statistics(S):
    t, reqs = S.make_trace(400, rate_hz=200.0, seed=6)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200.0) < 0.25 / 200.0
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 1000 and ns.max() <= 100000
    frac = np.mean([r.grad for r in reqs])
    assert 0.2 < frac < 0.4
    for r in reqs[:20]:
        assert r.z.max() - r.z.min() <= 0.5 + 1e-6 and r.z.max() <= 3.0 + 1e-6


def test_large_batch_evicts_idle_small_slots(S):
    # budget for one 400-slot; an idle 100-slot must be evicted to admit it
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 10}, budget_bytes=4000)
    p.enqueue(_Req(0, 80))
    take, b = p.next_batch("fwd")
    assert b == 100
    p.release("fwd", 100)
    p.enqueue(_Req(1, 350))
    take, b = p.next_batch("fwd")
    assert b == 400 and p.evicted == [("fwd", 100)] and p.reserved == 4000


def test_small_batch_reuses_idle_large_slot(S):
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 10}, budget_bytes=4000)
    p.enqueue(_Req(0, 350))
    p.next_batch("fwd")
    p.release("fwd", 400)
    p.enqueue(_Req(1, 50))
    take, b = p.next_batch("fwd")
    assert b == 400 and p.reserved == 4000 and not p.evicted

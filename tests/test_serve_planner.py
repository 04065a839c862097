"""Admission policy of the server (no GPU): the slot plan under an HBM
budget, FIFO batching into the allocated slots, per-kind lanes, the gradient
batch limit, timeouts and cancellation."""

import numpy as np
import pytest


class _Req:
    def __init__(self, rid, n, grad=False, t_submit=0.0, timeout_s=None):
        self.rid, self.n, self.grad, self.error = rid, n, grad, None
        self.t_submit, self.timeout_s, self.cancelled = t_submit, timeout_s, False

    @property
    def kind(self):
        return "grad" if self.grad else "fwd"


@pytest.fixture(scope="module")
def S():
    # importing the server touches no GPU (the binding only loads the library)
    import paper_2112_06830_amd.serve as S
    return S


def _planner(S, buckets=(100, 400), bpg=None, budget=10**9, slots=1, lanes=1, grad_cap=None):
    p = S.AdmissionPlanner(buckets, bpg or {"fwd": 10, "grad": 20}, budget, slots, lanes,
                           {"grad": grad_cap} if grad_cap else None)
    p.plan_slots()
    return p


def test_plan_takes_largest_bucket_of_each_kind_first(S):
    # the budget holds one 400-slot of each kind (4000 + 8000) and one more
    # 100-slot of fwd (1000): the largest sizes come first, then smallest first
    p = S.AdmissionPlanner([100, 400], {"fwd": 10, "grad": 20}, 13000, slots_per_bucket=2)
    new = p.plan_slots()
    assert new == [("fwd", 400), ("grad", 400), ("fwd", 100)]
    assert p.reserved == 13000 and p.reserved <= p.budget
    assert p.largest_slot("fwd") == 400 and p.largest_slot("grad") == 400


def test_plan_respects_slots_per_bucket(S):
    p = S.AdmissionPlanner([100, 400], {"fwd": 1, "grad": 1}, 10**9, slots_per_bucket=2)
    new = p.plan_slots()
    assert sorted(new) == sorted([("fwd", 100)] * 2 + [("fwd", 400)] * 2 +
                                 [("grad", 100)] * 2 + [("grad", 400)] * 2)
    assert p.plan_slots() == []                   # nothing more to add


def test_fifo_batches_fit_largest_idle_slot(S):
    p = _planner(S, lanes=2)
    for i, n in enumerate([50, 60, 200, 90, 30]):
        assert p.enqueue(_Req(i, n))
    take, bucket = p.next_batch("fwd")
    assert [r.rid for r in take] == [0, 1, 2, 3] and bucket == 400
    take2, bucket2 = p.next_batch("fwd")
    assert [r.rid for r in take2] == [4] and bucket2 == 100
    assert p.next_batch("fwd") is None


def test_busy_lanes_absorb_arrivals(S):
    # while the kind's one lane is busy, arrivals queue and leave together
    p = _planner(S)
    p.enqueue(_Req(0, 50))
    take, bucket = p.next_batch("fwd")
    assert [r.rid for r in take] == [0] and bucket == 100
    for i in range(1, 4):
        p.enqueue(_Req(i, 60))
    assert p.next_batch("fwd") is None            # the kind's lane is still busy
    p.enqueue(_Req(9, 10, grad=True))
    assert [r.rid for r in p.next_batch("grad")[0]] == [9]   # other kind unaffected
    p.release("fwd", 100)
    take, bucket = p.next_batch("fwd")
    assert [r.rid for r in take] == [1, 2, 3] and bucket == 400


def test_batch_waits_for_an_idle_slot_that_holds_it(S):
    # the only 400-slot is busy: a 350-galaxy request waits rather than
    # allocating, and a later small one does not overtake it (FIFO)
    p = _planner(S, lanes=2)
    p.enqueue(_Req(0, 300))
    assert p.next_batch("fwd")[1] == 400
    p.enqueue(_Req(1, 350))
    p.enqueue(_Req(2, 20))
    assert p.next_batch("fwd") is None
    assert p.reserved == 4000 + 1000 + 8000 + 2000      # unchanged: the loop never allocates
    p.release("fwd", 400)
    take, b = p.next_batch("fwd")
    assert [r.rid for r in take] == [1, 2] and b == 400  # 370 galaxies, in order


def test_batch_takes_smallest_idle_slot(S):
    p = _planner(S, lanes=2)
    p.enqueue(_Req(0, 80))
    assert p.next_batch("fwd")[1] == 100
    p.enqueue(_Req(1, 70))                        # the 100-slot is busy: the 400 one
    assert p.next_batch("fwd")[1] == 400


def test_gradient_batch_limit(S):
    # small gradient requests batch up to the limit; a large one goes alone
    p = _planner(S, buckets=(100, 400, 1600), slots=2, lanes=4, grad_cap=200)
    for i, n in enumerate([90, 80, 70, 1000, 60]):
        p.enqueue(_Req(i, n, grad=True))
    assert [r.rid for r in p.next_batch("grad")[0]] == [0, 1]          # 170 <= 200
    assert [r.rid for r in p.next_batch("grad")[0]] == [2]             # + 1000 > 200
    take, b = p.next_batch("grad")
    assert [r.rid for r in take] == [3] and b == 1600                  # alone
    assert [r.rid for r in p.next_batch("grad")[0]] == [4]
    # forward batches have no such limit
    for i, n in enumerate([90, 80, 70, 60]):
        p.enqueue(_Req(10 + i, n))
    assert len(p.next_batch("fwd")[0]) == 4


def test_oversize_request_rejected(S):
    p = _planner(S)
    r = _Req(0, 401)
    assert not p.enqueue(r) and "exceeds" in r.error
    # a budget that holds no slot of the request's kind admits nothing of it
    p2 = _planner(S, budget=4000)                 # one fwd 400-slot, no grad slot
    assert p2.enqueue(_Req(1, 350))
    r2 = _Req(2, 10, grad=True)
    assert not p2.enqueue(r2) and "exceeds" in r2.error


def test_timeouts_drop_requests_still_queued(S):
    p = _planner(S)
    p.enqueue(_Req(0, 50, t_submit=0.0))
    assert p.next_batch("fwd", now=0.0) is not None          # starts: no timeout applies
    p.enqueue(_Req(1, 50, t_submit=0.1, timeout_s=0.5))
    p.enqueue(_Req(2, 50, t_submit=0.2, timeout_s=5.0))
    p.enqueue(_Req(3, 50, t_submit=0.3))
    assert p.next_batch("fwd", now=1.0) is None              # lane busy; 1 has expired
    assert [r.rid for r in p.dropped] == [1] and "timed out" in p.dropped[0].error
    p.release("fwd", 100)
    take, _ = p.next_batch("fwd", now=1.1)
    assert [r.rid for r in take] == [2, 3]
    assert all(r.error is None for r in take)


def test_cancel_only_while_queued(S):
    p = _planner(S)
    a, b, c = _Req(0, 50), _Req(1, 50), _Req(2, 50)
    for r in (a, b, c):
        p.enqueue(r)
    take, _ = p.next_batch("fwd")
    assert take == [a, b, c]
    p.release("fwd", 400)
    d, e = _Req(3, 50), _Req(4, 50)
    p.enqueue(d)
    p.enqueue(e)
    assert not p.cancel(a)                        # already started
    assert p.cancel(d)
    take, _ = p.next_batch("fwd")
    assert take == [e]
    assert p.dropped == [d] and d.error == "cancelled"
    assert not p.cancel(_Req(9, 5))               # never queued


def test_kinds_queue_separately(S):
    p = _planner(S, buckets=(100,), bpg={"fwd": 1, "grad": 1})
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


def test_latency_summary_per_kind(S):
    _, reqs = S.make_trace(40, seed=8)
    lat = np.arange(40, dtype=np.float64)
    reqs[5].error = "timed out"
    out = S.latency_summary(reqs, 2.0, latencies_ms=lat)
    n_grad = sum(r.grad for i, r in enumerate(reqs) if i != 5)
    assert out["rejected"] == 1
    assert out["grad"]["requests"] == n_grad and out["fwd"]["requests"] == 39 - n_grad
    assert out["max_ms"] == 39.0

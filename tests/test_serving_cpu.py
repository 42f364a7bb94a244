"""Serving scheduler on the CPU: a fake executor with a virtual clock stands in
for the GPU (results from the CPU oracle), so admission, continuous batching
and per-request exactness are checked without a device."""
import numpy as np
import pytest

import synth
from oracle import lcp_oracle as O
from paper_2602_04936_amd import serve


class FakeExecutor:
    """Slots with a service time of a + b * queries (virtual seconds)."""

    def __init__(self, db, n_slots, cap_q, cap_e, a=2e-4, b=2e-6):
        self.db = db
        self.slots = [None] * n_slots
        self.now = 0.0
        self.a, self.b = a, b
        self.cap_q, self.cap_e = cap_q, cap_e
        self.launches = []

    def clock(self):
        return self.now

    def free_slot(self):
        for i, s in enumerate(self.slots):
            if s is None:
                return i
        return None

    def launch(self, slot, batch):
        nq = sum(r.b for r in batch)
        ne = sum(r.b * r.k for r in batch)
        assert nq <= self.cap_q and ne <= self.cap_e
        self.launches.append((self.now, [r.rid for r in batch]))
        for r in batch:
            ids = np.empty((r.b, r.k), np.int32)
            lcps = np.empty((r.b, r.k), np.int32)
            for j in range(r.b):
                ids[j], lcps[j] = O.topk(self.db, r.queries[j], r.k)
            r._pending = (ids, lcps)
        self.slots[slot] = (self.now + self.a + self.b * nq, batch)

    def poll(self, now_fn):
        done = []
        for i, s in enumerate(self.slots):
            if s is not None and s[0] <= self.now:
                for r in s[1]:
                    r.ids, r.lcps = r._pending
                    r.done = s[0]
                    done.append(r)
                self.slots[i] = None
        return done

    def busy(self):
        return any(s is not None for s in self.slots)

    def advance(self, next_arrival):
        cands = [s[0] for s in self.slots if s is not None]
        if next_arrival is not None:
            cands.append(next_arrival)
        if cands:
            self.now = max(self.now, min(cands))


def _workload(rate, seconds, k_mode="uniform", seed=3):
    rng = np.random.default_rng(seed)
    db = synth.random_rows(rng, 400, 6, 3)
    pool = np.concatenate([synth.random_rows(rng, 200, 6, 3), db[:50]])
    t, b, k = synth.serving_schedule(rate, seconds, seed=seed, k_mode=k_mode, k_fixed=7, max_batch=16)
    return db, serve.requests_from_schedule(pool, t, b, k)


def test_every_request_answered_exactly_as_alone():
    db, reqs = _workload(20000, 0.05)
    ex = FakeExecutor(db, n_slots=2, cap_q=64, cap_e=64 * 100)
    done = serve.run_loop(reqs, serve.Scheduler(64, 64 * 100), ex, clock=ex.clock)
    assert len(done) == len(reqs)
    for r in done:
        for j in range(r.b):
            ids, lcps = O.topk(db, r.queries[j], r.k)
            assert (r.ids[j] == ids).all() and (r.lcps[j] == lcps).all()
        assert r.done >= r.arrival + ex.a


def test_requests_arriving_during_a_launch_join_the_next_one():
    db, reqs = _workload(50000, 0.02)
    ex = FakeExecutor(db, n_slots=1, cap_q=256, cap_e=256 * 100, a=2e-3)
    serve.run_loop(reqs, serve.Scheduler(256, 256 * 100), ex, clock=ex.clock)
    sizes = [len(ids) for _, ids in ex.launches]
    assert max(sizes) > 1            # batching happened
    flat = [i for _, ids in ex.launches for i in ids]
    assert flat == sorted(flat)      # FIFO across launches
    assert sorted(flat) == [r.rid for r in sorted(reqs, key=lambda r: r.rid)]


def test_capacity_limits_are_respected():
    db, reqs = _workload(80000, 0.02)
    ex = FakeExecutor(db, n_slots=3, cap_q=20, cap_e=20 * 100)
    serve.run_loop(reqs, serve.Scheduler(20, 20 * 100), ex, clock=ex.clock)
    assert len(ex.launches) > 0


def test_request_larger_than_a_slot_is_rejected():
    s = serve.Scheduler(4, 40)
    with pytest.raises(ValueError):
        s.submit(serve.Request(0, 0.0, np.zeros((5, 3), np.uint8), 1))
    with pytest.raises(ValueError):
        s.submit(serve.Request(1, 0.0, np.zeros((4, 3), np.uint8), 11))


def test_slot_capacities_fit_the_budget():
    cq, ce = serve.slot_capacities(1 << 30, 3, 64, k_max=100)
    per = cq * (64 + 12) + ce * 8
    assert 3 * per <= 1 << 30 and cq > 0 and ce == cq * 100


def test_latency_report_fields():
    r = [serve.Request(i, 0.1 * i, np.zeros((2, 3), np.uint8), 1) for i in range(10)]
    for x in r:
        x.done = x.arrival + 0.001 * (1 + x.rid)
    rep = serve.latency_report(r, 1.0)
    assert rep["requests"] == 10 and rep["queries"] == 20
    assert rep["p50_ms"] == pytest.approx(5.5, abs=1e-9) and rep["p99_ms"] <= 10.0

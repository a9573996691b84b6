"""The serving loop's scheduling on the CPU, with a fake device.

The fake executor runs each graph of a batch through the CPU oracle (so the
results can be checked against the oracle alone) and sleeps to stand in for
device time.  It records the footprint of the batches running at once so the
HBM-budget invariant can be checked, and it can be told to fail any batch
holding a given request (a stand-in for a device-side error such as a weight
overflow).
"""
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle
from paper_2403_01261_amd.serve import Request, Scheduler, Server, footprint, poisson_arrivals, summarize


class FakeExecutor:
    def __init__(self, seconds_per_batch=0.01, poison=(), bad=()):
        self.dt = seconds_per_batch
        self.poison = set(poison)
        self.bad = set(bad)
        self.lock = threading.Lock()
        self.running_bytes = 0
        self.peak_bytes = 0
        self.calls = []

    def run(self, slot, batch):
        size = sum(r.bytes for r in batch)
        with self.lock:
            self.running_bytes += size
            self.peak_bytes = max(self.peak_bytes, self.running_bytes)
            self.calls.append((slot, [r.rid for r in batch], time.perf_counter()))
        try:
            time.sleep(self.dt)
            if self.poison & {r.rid for r in batch}:
                raise RuntimeError("device error in batch")
            out = []
            for r in batch:
                if r.rid in self.bad:
                    out.append((None, 0, -1))
                    continue
                res = oracle.lpa(r.payload)
                out.append((res.labels, res.iterations, 0))
            return out
        finally:
            with self.lock:
                self.running_bytes -= size


def make_requests(count, rate, seed=1, sizes=(20, 400)):
    rng = np.random.default_rng(seed)
    times = poisson_arrivals(count, rate, seed)
    reqs = []
    for k, t in enumerate(times):
        n = int(rng.integers(*sizes))
        g = graphgen.planted(n, max(2, n // 20), 0.3, n, 1000 + k)
        reqs.append(Request(rid=k, arrival=float(t), n=g.n, nnz=g.nnz, payload=g))
    return reqs


def check_against_oracle(reqs):
    for r in reqs:
        if r.state != "done":
            continue
        res = oracle.lpa(r.payload)
        np.testing.assert_array_equal(r.labels, res.labels)
        assert r.iterations == res.iterations


def test_footprint_formula():
    assert footprint(0, 0) == 64
    assert footprint(10, 100) == 64 * 11 + 400
    assert footprint(10, 100, weighted=True) == 64 * 11 + 800


def test_scheduler_fifo_budget_and_limits():
    s = Scheduler(budget_bytes=10_000, max_batch_graphs=2)
    reqs = [Request(rid=k, arrival=0.0, n=30, nnz=100) for k in range(5)]  # 2384 bytes each
    for r in reqs:
        assert s.submit(r)
    b1 = s.next_batch()
    assert [r.rid for r in b1] == [0, 1]          # batch size limit
    b2 = s.next_batch()
    assert [r.rid for r in b2] == [2, 3]          # FIFO
    assert s.next_batch() == []                   # 4 * 2384 + 2384 > 10000: wait for memory
    s.release(b1)
    assert [r.rid for r in s.next_batch()] == [4]
    assert s.peak_in_flight <= 10_000
    big = Request(rid=9, arrival=0.0, n=1000, nnz=10)
    assert not s.submit(big) and big.state == "rejected"


def test_all_requests_served_and_match_oracle():
    reqs = make_requests(60, rate=2000.0)
    ex = FakeExecutor(0.01)
    srv = Server(ex, slots=2, budget_bytes=1 << 30)
    srv.serve(reqs)
    assert all(r.state == "done" for r in reqs)
    check_against_oracle(reqs)
    summary = summarize(reqs, srv.batches)
    assert summary["done"] == 60
    assert summary["mean_batch"] > 1.0  # arrivals during a batch are batched together
    assert summary["p99_ms"] >= summary["p50_ms"] > 0


def test_budget_is_never_exceeded():
    reqs = make_requests(40, rate=5000.0, sizes=(200, 400))
    budget = 3 * max(r.bytes for r in reqs)
    ex = FakeExecutor(0.005)
    srv = Server(ex, slots=3, budget_bytes=budget)
    srv.serve(reqs)
    assert all(r.state == "done" for r in reqs)
    assert ex.peak_bytes <= budget
    assert srv.sched.peak_in_flight <= budget
    assert srv.sched.in_flight == 0


def test_oversize_request_rejected_alone():
    reqs = make_requests(10, rate=1000.0)
    huge = Request(rid=99, arrival=0.001, n=10 ** 6, nnz=10 ** 7, payload=None)
    srv = Server(FakeExecutor(0.002), slots=2, budget_bytes=1 << 20)
    srv.serve(reqs + [huge])
    assert huge.state == "rejected"
    assert all(r.state == "done" for r in reqs)
    check_against_oracle(reqs)


def test_failing_request_fails_alone():
    reqs = make_requests(30, rate=20000.0)  # bursty: batches of several requests
    ex = FakeExecutor(0.005, poison={7}, bad={11})
    srv = Server(ex, slots=2, budget_bytes=1 << 30)
    srv.serve(reqs)
    for r in reqs:
        if r.rid in (7, 11):
            assert r.state == "failed", r.rid
        else:
            assert r.state == "done", r.rid
    check_against_oracle(reqs)
    # the poisoned batch held other requests, which were rerun one by one
    assert any(7 in rids and len(rids) > 1 for _, rids, _ in ex.calls)


def test_cancel_queued_request():
    reqs = make_requests(12, rate=1e6)  # all arrive at once
    ex = FakeExecutor(0.02)
    srv = Server(ex, slots=1, budget_bytes=1 << 30, max_batch_graphs=2)
    srv.serve(reqs, cancel={0.005: [11]})
    assert reqs[11].state == "cancelled"
    assert not any(11 in rids for _, rids, _ in ex.calls)
    assert sum(r.state == "done" for r in reqs) == 11


def test_requests_admitted_while_others_run():
    # slot 0 is busy with the first batch when request 1 arrives: it must start
    # on slot 1 before the first batch ends (continuous batching, not a queue)
    reqs = make_requests(2, rate=1.0)
    reqs[0].arrival, reqs[1].arrival = 0.0, 0.01
    ex = FakeExecutor(0.1)
    srv = Server(ex, slots=2, budget_bytes=1 << 30)
    srv.serve(reqs)
    assert reqs[0].slot != reqs[1].slot
    assert reqs[1].t_admit < reqs[0].t_done


def test_poisson_arrivals():
    t = np.array(poisson_arrivals(20000, 2000.0, 3))
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert abs(np.diff(t).mean() - 0.0005) < 0.00002
    with pytest.raises(ValueError):
        Scheduler(0)

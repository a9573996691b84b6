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
from paper_2403_01261_amd.serve import (ContinuousServer, Request, Scheduler, Server, footprint, poisson_arrivals,
                                        summarize)


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


def lin_cost(n, nnz, weighted=False):
    """A stand-in cost for the scheduling tests (no library needed)."""
    return 64 * (n + 1) + 4 * nnz * (2 if weighted else 1)


def test_footprint_is_the_library_bound():
    """footprint() is gsl_graphs_bytes' growth for one graph plus its labels,
    grows with the graph and covers the arrays every batch holds per vertex
    and per entry (the GPU tests check it against what a batch allocates)."""
    import os
    import paper_2403_01261_amd as gsl
    if not os.path.exists(gsl.LIB_PATH):
        pytest.skip("libgsl_lpa.so not built")
    from paper_2403_01261_amd.serve import base_bytes
    b0 = gsl.gsl_graphs_bytes(0, 0, 0)
    assert base_bytes() == b0 > 0
    assert footprint(10, 100) == gsl.gsl_graphs_bytes(10, 100, 1) - b0 + 40
    assert footprint(10, 100, weighted=True) == footprint(10, 100) + 400
    assert gsl.gsl_graphs_bytes(-1, 0, 1) == -1
    # per vertex: at least the label, change/flag, list, split and graph-id
    # arrays and the gathered offsets; per entry: the gathered column
    assert footprint(10 ** 6, 0) - footprint(0, 0) >= 10 ** 6 * 40
    assert footprint(0, 10 ** 6) - footprint(0, 0) >= 4 * 10 ** 6
    rng = np.random.default_rng(5)
    for _ in range(200):
        n, e = int(rng.integers(0, 10 ** 6)), int(rng.integers(0, 10 ** 8))
        assert footprint(n + 1, e) > footprint(n, e) and footprint(n, e + 4097) > footprint(n, e)
    # one hub of 16 M entries: staging and partition records grow with it
    assert footprint(2, 1 << 24) > footprint(2, 1 << 23) * 1.9


def test_scheduler_fifo_budget_and_limits():
    s = Scheduler(budget_bytes=10_000, max_batch_graphs=2, cost=lin_cost)
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
    srv = Server(ex, slots=2, budget_bytes=1 << 30, cost=lin_cost)
    srv.serve(reqs)
    assert all(r.state == "done" for r in reqs)
    check_against_oracle(reqs)
    summary = summarize(reqs, srv.batches)
    assert summary["done"] == 60
    assert summary["mean_batch"] > 1.0  # arrivals during a batch are batched together
    assert summary["p99_ms"] >= summary["p50_ms"] > 0


def test_budget_is_never_exceeded():
    reqs = make_requests(40, rate=5000.0, sizes=(200, 400))
    budget = 3 * max(lin_cost(r.n, r.nnz) for r in reqs)
    ex = FakeExecutor(0.005)
    srv = Server(ex, slots=3, budget_bytes=budget, cost=lin_cost)
    srv.serve(reqs)
    assert all(r.state == "done" for r in reqs)
    assert ex.peak_bytes <= budget
    assert srv.sched.peak_in_flight <= budget
    assert srv.sched.in_flight == 0


def test_oversize_request_rejected_alone():
    reqs = make_requests(10, rate=1000.0)
    huge = Request(rid=99, arrival=0.001, n=10 ** 6, nnz=10 ** 7, payload=None)
    srv = Server(FakeExecutor(0.002), slots=2, budget_bytes=1 << 20, cost=lin_cost)
    srv.serve(reqs + [huge])
    assert huge.state == "rejected"
    assert all(r.state == "done" for r in reqs)
    check_against_oracle(reqs)


def test_failing_request_fails_alone():
    reqs = make_requests(30, rate=20000.0)  # bursty: batches of several requests
    ex = FakeExecutor(0.005, poison={7}, bad={11})
    srv = Server(ex, slots=2, budget_bytes=1 << 30, cost=lin_cost)
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
    srv = Server(ex, slots=1, budget_bytes=1 << 30, max_batch_graphs=2, cost=lin_cost)
    srv.serve(reqs, cancel={0.005: [11]})
    assert reqs[11].state == "cancelled"
    assert not any(11 in rids for _, rids, _ in ex.calls)
    assert sum(r.state == "done" for r in reqs) == 11


def test_requests_admitted_while_others_run():
    # slot 0 is busy with the first batch when request 1 arrives: it must start
    # on slot 1 before the first batch ends (continuous batching, not a queue)
    reqs = make_requests(2, rate=1.0)
    # arrivals 0.1 s apart: the server's first look at the queue may come late
    # on a loaded machine, and both requests must not be there yet
    reqs[0].arrival, reqs[1].arrival = 0.0, 0.1
    ex = FakeExecutor(1.0)
    srv = Server(ex, slots=2, budget_bytes=1 << 30, cost=lin_cost)
    srv.serve(reqs)
    assert reqs[0].slot != reqs[1].slot
    assert reqs[1].t_admit < reqs[0].t_done


def test_poisson_arrivals():
    t = np.array(poisson_arrivals(20000, 2000.0, 3))
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert abs(np.diff(t).mean() - 0.0005) < 0.00002
    with pytest.raises(ValueError):
        Scheduler(0)


class FakeSession:
    """A session on the CPU: graphs take vertex / entry / slot capacity while
    they run, every step advances each running graph by `sweeps` sweeps, and
    a graph leaves with the oracle's labels once it has run the oracle's
    number of sweeps.  Records what was resident at every step."""

    def __init__(self, cap_v, cap_e, cap_g, seconds_per_step=0.002, poison=()):
        self.cap_v, self.cap_e, self.cap_g = cap_v, cap_e, cap_g
        self.dt = seconds_per_step
        self.poison = set(poison)  # a step holding one of these fails (a weight overflow)
        self.live = {}          # ticket -> [request, sweeps done, sweeps needed, labels]
        self.next = 0
        self.steps = []         # sets of resident request ids, per step
        self.resets = 0
        self.add_calls = []     # graphs offered per add call

    def _used(self):
        return (sum(r.n for r, *_ in self.live.values()), sum(r.nnz for r, *_ in self.live.values()))

    def add(self, reqs):
        self.add_calls.append(len(reqs))
        out = []
        for r in reqs:
            if r.n > self.cap_v or r.nnz > self.cap_e:
                out.append((-1, -1))
                continue
            v, e = self._used()
            if len(self.live) >= self.cap_g or v + r.n > self.cap_v or e + r.nnz > self.cap_e:
                out.append((-1, ContinuousServer.EAGAIN))
                break
            if r.n == 0:
                out.append((-1, 0))
                continue
            res = oracle.lpa(r.payload)
            self.live[self.next] = [r, 0, res.iterations, res.labels]
            out.append((self.next, 0))
            self.next += 1
        return out

    def step(self, sweeps):
        time.sleep(self.dt)
        self.steps.append({x[0].rid for x in self.live.values()})
        if self.poison & self.steps[-1]:
            err = RuntimeError("a row's summed weight reaches 2^32")
            err.code = -4
            raise err
        done = []
        for t, x in list(self.live.items()):
            x[1] = min(x[1] + sweeps, x[2])
            if x[1] >= x[2]:
                x[0].labels = x[3]
                done.append((t, x[2]))
                del self.live[t]
        return done

    def collect(self, r):
        pass

    def reset(self):
        self.live.clear()
        self.resets += 1

    def room(self):
        v, e = self._used()
        return self.cap_v - v, self.cap_e - e, self.cap_g - len(self.live)

    def live_count(self):
        return len(self.live)


def test_continuous_server_admits_between_sweeps_and_matches_oracle():
    reqs = make_requests(50, rate=3000.0)
    fs = FakeSession(cap_v=2000, cap_e=40_000, cap_g=8)
    srv = ContinuousServer(fs, sweeps_per_step=1)
    srv.serve(reqs)
    assert all(r.state == "done" for r in reqs)
    check_against_oracle(reqs)
    # requests joined batches that were already running (continuous batching)
    joined = any(len(a - b) > 0 and len(a & b) > 0 for b, a in zip(fs.steps, fs.steps[1:]))
    assert joined
    assert max(len(s) for s in fs.steps) <= 8
    assert summarize(reqs)["done"] == 50


def test_continuous_server_capacity_retry_and_rejection():
    reqs = make_requests(30, rate=1e6, sizes=(300, 400))   # all at once, more than fits
    huge = Request(rid=999, arrival=0.0, n=10 ** 6, nnz=10, payload=None)
    fs = FakeSession(cap_v=1000, cap_e=10 ** 6, cap_g=64)
    srv = ContinuousServer(fs, sweeps_per_step=2)
    srv.serve(reqs + [huge])
    assert huge.state == "failed"
    assert all(r.state == "done" for r in reqs)
    check_against_oracle(reqs)
    # never more resident vertices than the capacity
    by_rid = {r.rid: r for r in reqs}
    assert all(sum(by_rid[i].n for i in s) <= 1000 for s in fs.steps)
    # later requests waited for earlier ones to leave
    assert min(r.t_admit for r in reqs[-5:]) > 0
    # the server offers only what the free capacity can hold (three graphs of
    # 300-400 vertices at most here), not a long slice of the queue each step
    assert max(fs.add_calls) <= 3


def test_continuous_server_cancel():
    reqs = make_requests(20, rate=1e6)
    fs = FakeSession(cap_v=500, cap_e=10 ** 6, cap_g=2, seconds_per_step=0.005)
    srv = ContinuousServer(fs, sweeps_per_step=1)
    srv.serve(reqs, cancel={0.002: [19]})
    assert reqs[19].state == "cancelled"
    assert sum(r.state == "done" for r in reqs) == 19


def test_continuous_server_failing_step_fails_only_the_culprit():
    """A step that fails loses every graph it held; the server resets the
    session and runs those requests again one at a time, so only the culprit
    fails (with the library's code) and the others match the oracle."""
    reqs = make_requests(40, rate=20000.0)  # bursty: many graphs per step
    fs = FakeSession(cap_v=4000, cap_e=10 ** 6, cap_g=16, poison={12})
    srv = ContinuousServer(fs, sweeps_per_step=1)
    srv.serve(reqs)
    assert reqs[12].state == "failed" and reqs[12].code == -4
    assert all(r.state == "done" for r in reqs if r.rid != 12)
    check_against_oracle(reqs)
    assert srv.failed_steps >= 2 and fs.resets == srv.failed_steps
    # the failed step held others besides the culprit, and the culprit's last
    # step held it alone
    failed = [st for st in fs.steps if 12 in st]
    assert len(failed[0]) > 1 and failed[-1] == {12}

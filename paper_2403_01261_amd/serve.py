"""Serving loop: continuous batching of community-detection requests.

A request carries one graph already resident in device memory (CSR tensors
the client uploaded).  Requests arrive over time.  A dispatcher keeps a FIFO
queue and a set of slots; a slot is a worker thread that owns a gsl_context
(its own scratch and stream).  Whenever a slot is idle, the dispatcher admits
requests from the head of the queue into one batch, as many as the HBM budget
and the batch limits allow, and hands the batch to the slot, which runs it as
one gsl_lpa_graphs call.  Requests that arrive meanwhile wait for the next
idle slot, so batches of different slots overlap on the device, and a new
request never waits for a whole earlier batch to drain unless every slot is
busy or the budget is spent.

Admission is by device-memory footprint (footprint()): the library's bound
of the scratch a batch needs for the graph (gsl_graphs_bytes), plus the
labels; each slot's fixed scratch comes off the budget once.  The sum over
admitted, unfinished requests never exceeds the budget; a request whose own
footprint exceeds it is rejected at once.  Errors stay with their
request: gsl_lpa_graphs reports a malformed graph on its own (status
GSL_EINVAL), and if a whole batch fails (for instance a weight overflow), the
slot reruns its requests one by one so only the culprit fails.

The scheduling logic (Scheduler, Server) is plain Python and takes the
executor as a parameter, so it is tested on the CPU with a fake executor; the
GPU executor is GpuExecutor.  PlainExecutor runs one gsl_lpa call per
request, the baseline the batched server is compared with.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Any, Callable, List, Optional

def footprint(n: int, nnz: int, weighted: bool = False) -> int:
    """Device bytes a request adds to a batch while it runs, from the
    library's own bound (gsl_graphs_bytes): what a batch holding this graph
    needs beyond an empty batch, plus the request's 4-byte output labels.  The
    bound's terms grow no faster than linearly with a batch's totals, except
    the hub tier's, which is bounded per graph; so the footprints of a
    batch's graphs plus base_bytes() bound the batch."""
    from . import gsl_graphs_bytes
    return gsl_graphs_bytes(n, nnz, 1, weighted) - gsl_graphs_bytes(0, 0, 0, weighted) + 4 * n


def base_bytes(weighted: bool = False) -> int:
    """Scratch of an empty batch (counters, per-tier records, partials): held
    once per slot."""
    from . import gsl_graphs_bytes
    return gsl_graphs_bytes(0, 0, 0, weighted)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float              # seconds after the start of the stream
    n: int
    nnz: int
    weighted: bool = False
    payload: Any = None         # what the executor needs (device tensors, or a CPU graph in tests)
    # filled in by the server
    state: str = "new"          # new, queued, running, done, failed, rejected, cancelled
    code: int = 0               # gsl_status of a failed request
    error: str = ""
    t_admit: float = float("nan")
    t_done: float = float("nan")
    slot: int = -1
    batch_id: int = -1
    labels: Any = None
    iterations: int = -1
    cost: int = -1              # device bytes charged to the budget (set by the scheduler)

    @property
    def bytes(self) -> int:
        return self.cost if self.cost >= 0 else footprint(self.n, self.nnz, self.weighted)

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


class Scheduler:
    """FIFO admission under a device-memory budget (no GPU involved).
    `cost(n, nnz, weighted)` gives a request's device bytes (footprint() by
    default)."""

    def __init__(self, budget_bytes: int, max_batch_graphs: int = 1024, max_batch_bytes: Optional[int] = None,
                 cost: Optional[Callable[[int, int, bool], int]] = None):
        if budget_bytes <= 0 or max_batch_graphs <= 0:
            raise ValueError("budget and batch size must be positive")
        self.cost = cost or footprint
        self.budget = int(budget_bytes)
        self.max_graphs = int(max_batch_graphs)
        self.max_bytes = int(max_batch_bytes) if max_batch_bytes else self.budget
        self.queue: collections.deque = collections.deque()
        self.in_flight = 0
        self.peak_in_flight = 0

    def submit(self, req: Request) -> bool:
        req.cost = int(self.cost(req.n, req.nnz, req.weighted))
        if req.bytes > min(self.budget, self.max_bytes):
            req.state = "rejected"
            req.code = -2  # GSL_ENOMEM: can never fit
            req.error = "footprint %d bytes exceeds the budget" % req.bytes
            return False
        req.state = "queued"
        self.queue.append(req)
        return True

    def cancel(self, rid: int) -> bool:
        for r in self.queue:
            if r.rid == rid:
                self.queue.remove(r)
                r.state = "cancelled"
                return True
        return False

    def next_batch(self) -> List[Request]:
        """Requests from the head of the queue that fit now (possibly none)."""
        batch, size = [], 0
        while self.queue and len(batch) < self.max_graphs:
            b = self.queue[0].bytes
            if self.in_flight + size + b > self.budget or size + b > self.max_bytes:
                break
            batch.append(self.queue.popleft())
            size += b
        self.in_flight += size
        self.peak_in_flight = max(self.peak_in_flight, self.in_flight)
        return batch

    def release(self, batch: List[Request]) -> None:
        self.in_flight -= sum(r.bytes for r in batch)


class Server:
    """Continuous-batching request loop over `slots` worker threads.

    executor.run(slot, batch) returns one (labels, iterations, status) per
    request of the batch or raises; status 0 is success."""

    def __init__(self, executor, slots: int = 2, budget_bytes: int = 32 << 30, max_batch_graphs: int = 1024,
                 max_batch_bytes: Optional[int] = None, clock: Callable[[], float] = time.perf_counter,
                 cost: Optional[Callable[[int, int, bool], int]] = None, slot_base_bytes: Optional[int] = None):
        """cost: a request's device bytes (footprint() by default);
        slot_base_bytes: what each slot holds with an empty batch, taken off
        the budget once per slot (base_bytes(True) by default, 0 with a
        custom cost)."""
        if slots <= 0:
            raise ValueError("slots must be positive")
        self.executor = executor
        self.slots = slots
        if slot_base_bytes is None:
            slot_base_bytes = 0 if cost is not None else base_bytes(True)
        budget = int(budget_bytes) - slots * int(slot_base_bytes)
        if budget <= 0:
            raise ValueError("the budget does not cover the slots' fixed scratch (%d bytes each)" % slot_base_bytes)
        self.sched = Scheduler(budget, max_batch_graphs, max_batch_bytes, cost)
        self.clock = clock
        self.batches: List[List[Request]] = []

    def _work(self, slot: int, inbox: queue.Queue, done: queue.Queue, t0: float):
        while True:
            batch = inbox.get()
            if batch is None:
                return
            try:
                out = self.executor.run(slot, batch)
                t = self.clock() - t0
                for r, (lab, it, st) in zip(batch, out):
                    self._finish(r, lab, it, st, t)
            except Exception as e:  # the whole batch failed: isolate the culprit
                if len(batch) == 1:
                    self._fail(batch[0], e, self.clock() - t0)
                else:
                    for r in batch:
                        try:
                            (lab, it, st), = self.executor.run(slot, [r])
                            self._finish(r, lab, it, st, self.clock() - t0)
                        except Exception as e1:
                            self._fail(r, e1, self.clock() - t0)
            done.put((slot, batch))

    @staticmethod
    def _finish(r: Request, lab, it, st, t):
        r.t_done = t
        if st == 0:
            r.state, r.labels, r.iterations = "done", lab, it
        else:
            r.state, r.code, r.error = "failed", st, "graph rejected by the library"

    @staticmethod
    def _fail(r: Request, e: Exception, t):
        r.t_done = t
        r.state = "failed"
        r.code = getattr(e, "code", -3)
        r.error = str(e)

    def serve(self, requests: List[Request], cancel: Optional[dict] = None) -> List[Request]:
        """Runs the stream to completion.  `cancel` maps a time (s) to request
        ids cancelled at that moment if still queued."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque(reqs)
        cancels = sorted((cancel or {}).items())
        inboxes = [queue.Queue() for _ in range(self.slots)]
        done: queue.Queue = queue.Queue()
        t0 = self.clock()
        workers = [threading.Thread(target=self._work, args=(s, inboxes[s], done, t0), daemon=True)
                   for s in range(self.slots)]
        for w in workers:
            w.start()
        idle = list(range(self.slots))
        busy = 0
        try:
            while pending or self.sched.queue or busy:
                now = self.clock() - t0
                while pending and pending[0].arrival <= now:
                    self.sched.submit(pending.popleft())
                while cancels and cancels[0][0] <= now:
                    for rid in cancels.pop(0)[1]:
                        self.sched.cancel(rid)
                while idle and self.sched.queue:
                    batch = self.sched.next_batch()
                    if not batch:
                        break
                    slot = idle.pop(0)
                    t = self.clock() - t0
                    for r in batch:
                        r.state, r.t_admit, r.slot, r.batch_id = "running", t, slot, len(self.batches)
                    self.batches.append(batch)
                    busy += 1
                    inboxes[slot].put(batch)
                # wait for a completion or the next arrival / cancellation
                nxt = [pending[0].arrival] if pending else []
                if cancels:
                    nxt.append(cancels[0][0])
                wait = 0.05 if not nxt else max(0.0, min(nxt) - (self.clock() - t0))
                if busy == 0 and not nxt:
                    # queued work that cannot be admitted with nothing in flight
                    if self.sched.queue:
                        raise RuntimeError("queued requests can never be admitted")
                    break
                try:
                    item = done.get(timeout=min(wait, 0.002) if busy else wait)
                except queue.Empty:
                    continue
                while True:
                    slot, batch = item
                    self.sched.release(batch)
                    idle.append(slot)
                    busy -= 1
                    try:
                        item = done.get_nowait()
                    except queue.Empty:
                        break
        finally:
            for ib in inboxes:
                ib.put(None)
            for w in workers:
                w.join()
        return reqs


class ContinuousServer:
    """Continuous batching at sweep granularity over one resident batch (a
    gsl_session).  The loop alternates two things: admit queued requests, in
    arrival order, as far as the session's free vertices, entries and graph
    slots allow; run a step of a few sweeps of every admitted graph, after
    which the graphs that stopped leave with their labels.  A request that
    arrives while others run joins them at the next step instead of waiting
    for a batch to drain, and its result is what it would get alone (each
    graph keeps its own sweeps and convergence test in the session).

    A step that fails (a weight overflow fails the whole session) loses the
    graphs it held: the backend is reset and those requests run again one at
    a time, each alone in the session, so only the culprit fails.

    backend.add(requests) returns one (ticket, status) per request (status 0:
    admitted, ticket -1 when nothing has to run; EAGAIN: no room now, and the
    later requests of the call were not tried; anything else: rejected),
    backend.step(sweeps) returns [(ticket, sweeps_run)] of finished graphs or
    raises, backend.reset() empties the session after a failed step, and
    backend.room() (optional) gives the free (vertices, entries, graphs).
    Plain Python, tested on the CPU with a fake backend; SessionBackend is the
    GPU one."""

    EAGAIN = -5

    def __init__(self, backend, sweeps_per_step: int = 2, max_admit: int = 256,
                 clock: Callable[[], float] = time.perf_counter):
        if sweeps_per_step < 1 or max_admit < 1:
            raise ValueError("sweeps_per_step and max_admit must be positive")
        self.backend = backend
        self.sweeps = int(sweeps_per_step)
        self.max_admit = int(max_admit)
        self.clock = clock
        self.steps = 0
        self.admissions: List[int] = []   # requests admitted before each step
        self.failed_steps = 0

    def _admit(self, queue, by_ticket, suspects, t0) -> int:
        """Admits from the head of the queue; returns how many now run.  A
        suspect (it shared a failed step) runs only in an empty session and
        keeps the session to itself."""
        admitted = 0
        room = getattr(self.backend, "room", None)
        while queue:
            if any(r.rid in suspects for r in by_ticket.values()):
                break
            # as many as the session's free capacity can hold (the first is
            # always tried: it may be rejected outright), so a long queue does
            # not cost a table of max_admit graphs every step
            fv, fe, fg = room() if room else (float("inf"),) * 3
            head = []
            for k in range(min(len(queue), self.max_admit)):
                r = queue[k]
                if r.rid in suspects:
                    if not head and not by_ticket:
                        head = [r]
                    break
                if head and (r.n > fv or r.nnz > fe or fg < 1):
                    break
                head.append(r)
                fv, fe, fg = fv - r.n, fe - r.nnz, fg - 1
            if not head:
                break
            res = self.backend.add(head)
            stop = False
            t = self.clock() - t0
            for r, (ticket, status) in zip(head, res):
                if status == self.EAGAIN:
                    stop = True
                    break
                queue.popleft()
                r.t_admit = t
                if status != 0:
                    r.state, r.code, r.error, r.t_done = "failed", status, "graph rejected by the library", t
                elif ticket < 0:
                    r.state, r.iterations, r.t_done = "done", 0, t
                else:
                    r.state = "running"
                    by_ticket[ticket] = r
                    admitted += 1
            if stop or len(res) < len(head):
                break
        return admitted

    def serve(self, requests: List[Request], cancel: Optional[dict] = None) -> List[Request]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque(reqs)
        queue: collections.deque = collections.deque()
        cancels = sorted((cancel or {}).items())
        by_ticket = {}
        suspects = set()
        t0 = self.clock()
        while pending or queue or by_ticket:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                r.state = "queued"
                queue.append(r)
            while cancels and cancels[0][0] <= now:
                for rid in cancels.pop(0)[1]:
                    for r in list(queue):
                        if r.rid == rid:
                            queue.remove(r)
                            r.state = "cancelled"
            admitted = self._admit(queue, by_ticket, suspects, t0)
            if by_ticket:
                self.admissions.append(admitted)
                try:
                    finished = self.backend.step(self.sweeps)
                except Exception as e:  # the session's graphs are lost
                    self.failed_steps += 1
                    running = sorted(by_ticket.values(), key=lambda q: (q.arrival, q.rid))
                    by_ticket.clear()
                    self.backend.reset()
                    t = self.clock() - t0
                    if len(running) == 1 and running[0].rid in suspects:
                        r = running[0]
                        r.state, r.code, r.error, r.t_done = "failed", getattr(e, "code", -3), str(e), t
                    else:
                        for r in reversed(running):  # back to the head of the queue, in order
                            suspects.add(r.rid)
                            r.state = "queued"
                            queue.appendleft(r)
                    continue
                self.steps += 1
                t = self.clock() - t0
                for ticket, iters in finished:
                    r = by_ticket.pop(ticket)
                    r.state, r.iterations, r.t_done = "done", iters, t
                    self.backend.collect(r)
            elif pending:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
            elif queue:
                raise RuntimeError("queued requests can never be admitted")
        return reqs


class SessionBackend:
    """ContinuousServer backend on one gsl_session.  A request's payload is
    (offsets, cols, weights or None) device tensors with local ids; its labels
    land in a tensor of its own (request.labels)."""

    def __init__(self, max_vertices: int, max_entries: int, max_graphs: int = 4096, max_iters: int = 20,
                 tolerance: float = 0.05, weighted: bool = False):
        from . import Session
        self._args = (max_vertices, max_entries, max_graphs, max_iters, tolerance, weighted)
        self.session = Session(*self._args)

    def add(self, reqs):
        res = self.session.add([tuple(r.payload[:3]) for r in reqs])
        out = []
        for r, (ticket, status, lab) in zip(reqs, res):
            if status == 0:
                r.labels = lab
            out.append((ticket, status))
        return out

    def step(self, sweeps: int):
        return self.session.step(sweeps)

    def collect(self, r):
        pass

    def live(self) -> int:
        return self.session.info()["live_graphs"]

    def room(self):
        """Free vertices, entries and graph slots of the session."""
        i = self.session.info()
        return i["free_vertices"], i["free_entries"], self.session.max_graphs - i["live_graphs"]

    def reset(self):
        """A new, empty session in place of one whose step failed."""
        from . import Session
        self.session.close()
        self.session = Session(*self._args)

    def close(self):
        self.session.close()


def summarize(reqs: List[Request], batches: Optional[List[List[Request]]] = None) -> dict:
    """Latency percentiles (ms), throughput (graphs/s from the first arrival
    to the last completion) and outcome counts."""
    import numpy as np
    ok = [r for r in reqs if r.state == "done"]
    lat = np.array([r.latency for r in ok]) * 1e3 if ok else np.zeros(0)
    span = (max(r.t_done for r in ok) - min(r.arrival for r in reqs)) if ok else float("nan")
    out = {"requests": len(reqs), "done": len(ok),
           "failed": sum(r.state == "failed" for r in reqs),
           "rejected": sum(r.state == "rejected" for r in reqs),
           "cancelled": sum(r.state == "cancelled" for r in reqs),
           "graphs_per_s": len(ok) / span if ok and span > 0 else float("nan"),
           "p50_ms": float(np.percentile(lat, 50)) if ok else float("nan"),
           "p99_ms": float(np.percentile(lat, 99)) if ok else float("nan"),
           "mean_ms": float(lat.mean()) if ok else float("nan")}
    if batches is not None:
        out["batches"] = len(batches)
        out["mean_batch"] = (sum(len(b) for b in batches) / len(batches)) if batches else 0.0
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> List[float]:
    """Arrival times (s) of a Poisson stream: exponential gaps of mean 1/rate."""
    import numpy as np
    gaps = np.random.default_rng(seed).exponential(1.0 / rate_per_s, size=count)
    return list(np.cumsum(gaps) - gaps[0])


class GpuExecutor:
    """Runs a batch as one gsl_lpa_graphs call on the slot's own context."""

    def __init__(self, slots: int, max_iters: int = 20, tolerance: float = 0.05):
        from . import Context
        self.ctx = [Context() for _ in range(slots)]
        self.max_iters, self.tol = max_iters, tolerance

    def run(self, slot: int, batch: List[Request]):
        outs, iters, _, status = self.ctx[slot].lpa_graphs([r.payload for r in batch], self.max_iters, self.tol,
                                                           return_status=True)
        return list(zip(outs, iters, status))

    def close(self):
        for c in self.ctx:
            c.close()


class PlainExecutor:
    """One gsl_lpa call per request (payload: local-offset CSR tensors)."""

    def __init__(self, max_iters: int = 20, tolerance: float = 0.05):
        self.max_iters, self.tol = max_iters, tolerance

    def run(self, slot: int, batch: List[Request]):
        from . import gsl_lpa_ex
        res = []
        for r in batch:
            off, cols, w = r.payload[:3]
            lab, st = gsl_lpa_ex(off, cols, w, self.max_iters, self.tol)
            res.append((lab, st["iterations"], 0))
        return res

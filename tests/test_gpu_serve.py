"""The served path on the GPU: a Poisson stream of requests through the
continuous-batching server (two slots, each with its own context) gives every
request exactly the labels and sweep count it gets alone (gsl_lpa) and from
the oracle; a malformed graph and a weight overflow fail alone."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import graphgen  # noqa: E402
import oracle  # noqa: E402
from graphgen import workloads  # noqa: E402
from tests.gpu_util import say, to_device  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_01261_amd as m
    m.load()
    return m


def test_served_results_equal_alone_and_oracle(gsl):
    from paper_2403_01261_amd.serve import GpuExecutor, Request, Server, poisson_arrivals, summarize
    b = workloads.make(5, small=True)
    graphs = [b.subgraph(k) for k in range(b.num_graphs)]
    # edge cases mixed in: an isolated-only graph, a graph with a column out of
    # range, and one whose weights overflow 32 bits
    graphs.insert(5, graphgen.from_entries(4, [], []))
    bad = graphgen.from_undirected(6, [(0, 1), (1, 2)])
    graphs.insert(9, bad)
    ovf = graphgen.from_undirected(3, [(0, 1), (0, 2)], [1 << 31, 1 << 31])
    graphs.insert(13, ovf)
    times = poisson_arrivals(len(graphs), 2000.0, 7)
    reqs = []
    for k, (g, t) in enumerate(zip(graphs, times)):
        off, cols, w = to_device(g)
        if k == 9:
            cols = cols.clone()
            cols[0] = 17  # outside [0, 6)
        reqs.append(Request(rid=k, arrival=float(t), n=g.n, nnz=g.nnz, weighted=w is not None,
                            payload=(off, cols, w)))
    torch.cuda.synchronize()
    ex = GpuExecutor(2)
    srv = Server(ex, slots=2, budget_bytes=1 << 30)
    try:
        srv.serve(reqs)
    finally:
        ex.close()
    s = summarize(reqs, srv.batches)
    say("served:", s)
    assert reqs[9].state == "failed" and reqs[9].code == gsl.GSL_EINVAL
    assert reqs[13].state == "failed" and reqs[13].code == gsl.GSL_EOVERFLOW
    for k, (g, r) in enumerate(zip(graphs, reqs)):
        if k in (9, 13):
            continue
        assert r.state == "done", (k, r.state, r.error)
        exp = oracle.lpa(g)
        lab = r.labels.cpu().numpy()
        np.testing.assert_array_equal(lab, exp.labels, err_msg="request %d" % k)
        assert r.iterations == exp.iterations
        off, cols, w = r.payload
        alone, st = gsl.gsl_lpa_ex(off, cols, w)
        np.testing.assert_array_equal(lab, alone.cpu().numpy())
        assert st["iterations"] == r.iterations
    assert s["done"] == len(graphs) - 2


def test_continuous_server_requests_join_running_graphs(gsl):
    """Sweep-level continuous batching (ContinuousServer over a gsl_session):
    requests arriving while others run join them at the next step; every
    result equals gsl_lpa alone and the oracle, and a malformed graph fails
    alone."""
    from paper_2403_01261_amd.serve import ContinuousServer, Request, SessionBackend, poisson_arrivals, summarize
    b = workloads.make(5, small=True)
    graphs = [b.subgraph(k) for k in range(b.num_graphs)]
    graphs.insert(5, graphgen.from_entries(4, [], []))
    graphs.insert(9, graphgen.from_undirected(6, [(0, 1), (1, 2)]))
    times = poisson_arrivals(len(graphs), 2000.0, 11)
    reqs = []
    for k, (g, t) in enumerate(zip(graphs, times)):
        off, cols, w = to_device(g)
        if k == 9:
            cols = cols.clone()
            cols[0] = 17  # outside [0, 6)
        reqs.append(Request(rid=k, arrival=float(t), n=g.n, nnz=g.nnz, payload=(off, cols, w)))
    torch.cuda.synchronize()
    backend = SessionBackend(max_vertices=150_000, max_entries=3_000_000, max_graphs=32)
    srv = ContinuousServer(backend, sweeps_per_step=1)
    try:
        srv.serve(reqs)
    finally:
        backend.close()
    s = summarize(reqs)
    say("continuous:", s, "steps", srv.steps)
    assert reqs[9].state == "failed" and reqs[9].code == gsl.GSL_EINVAL
    # some request was admitted while earlier ones were still running
    running_at_admit = [sum(1 for q in reqs if q.t_admit < r.t_admit < q.t_done) for r in reqs if r.state == "done"]
    assert max(running_at_admit) > 0
    for k, (g, r) in enumerate(zip(graphs, reqs)):
        if k == 9:
            continue
        assert r.state == "done", (k, r.state, r.error)
        exp = oracle.lpa(g)
        lab = r.labels.cpu().numpy()
        np.testing.assert_array_equal(lab, exp.labels, err_msg="request %d" % k)
        assert r.iterations == exp.iterations
        off, cols, w = r.payload
        alone, st = gsl.gsl_lpa_ex(off, cols, w)
        np.testing.assert_array_equal(lab, alone.cpu().numpy())


def test_footprints_bound_what_the_library_allocates(gsl):
    """The serving budget's bytes are real: a fresh context running a batch of
    graphs, and a session with its graphs running, take no more device memory
    than the library's bounds (footprints plus the empty batch; the session's
    device_bytes) allow, up to allocation granularity."""
    from paper_2403_01261_amd.serve import base_bytes, footprint
    b = workloads.make(5, small=True)
    graphs = [b.subgraph(k) for k in range(b.num_graphs)]
    tens = [to_device(g)[:2] + (None, torch.empty(g.n, dtype=torch.int32, device="cuda")) for g in graphs]
    slack = 32 << 20
    bound = base_bytes() + sum(footprint(g.n, g.nnz) for g in graphs)
    with gsl.Context() as ctx:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        labs, its, _ = ctx.lpa_graphs(tens)
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info()[0]
    say("batch of %d graphs: %d bytes allocated, bound %d" % (len(graphs), used, bound))
    assert used <= bound + slack
    for g, lab in zip(graphs[:4], labs[:4]):
        np.testing.assert_array_equal(lab.cpu().numpy(), oracle.lpa(g).labels)
    cap_v, cap_e, cap_g = 1 << 20, 1 << 24, 64
    sbound = gsl.Session.device_bytes(cap_v, cap_e, cap_g)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    with gsl.Session(cap_v, cap_e, cap_g) as sess:
        got = sess.add(tens[:30])
        live = {t for t, st, _ in got if t >= 0}
        while live:
            live -= {t for t, _ in sess.step(2)}
        used = free0 - torch.cuda.mem_get_info()[0]
        assert sess.info()["device_bytes"] == sbound
    say("session: %d bytes allocated, bound %d" % (used, sbound))
    assert used <= sbound + slack


def test_continuous_server_weight_overflow_fails_alone(gsl):
    """A graph whose row weights sum to 2^32 makes its session step fail
    (GSL_EOVERFLOW) and loses the session's graphs; the continuous server
    starts a new session and reruns them one at a time, so only that graph
    fails and every other result still equals the oracle."""
    from paper_2403_01261_amd.serve import ContinuousServer, Request, SessionBackend
    b = workloads.make(5, small=True)
    graphs = [b.subgraph(k) for k in range(12)]
    ovf = graphgen.from_undirected(3, [(0, 1), (0, 2)], [1 << 31, 1 << 31])
    graphs.insert(4, ovf)
    reqs = []
    for k, g in enumerate(graphs):
        off, cols, _ = to_device(g)
        w = torch.from_numpy((g.weights if g.weights is not None else np.ones(g.nnz, np.uint32)).view(np.int32))
        reqs.append(Request(rid=k, arrival=0.0, n=g.n, nnz=g.nnz, weighted=True, payload=(off, cols, w.cuda())))
    torch.cuda.synchronize()
    backend = SessionBackend(max_vertices=150_000, max_entries=3_000_000, max_graphs=32, weighted=True)
    srv = ContinuousServer(backend, sweeps_per_step=2)
    try:
        srv.serve(reqs)
    finally:
        backend.close()
    say("failed steps", srv.failed_steps)
    assert reqs[4].state == "failed" and reqs[4].code == gsl.GSL_EOVERFLOW
    assert srv.failed_steps >= 2
    for k, (g, r) in enumerate(zip(graphs, reqs)):
        if k == 4:
            continue
        assert r.state == "done", (k, r.state, r.error)
        exp = oracle.lpa(g)
        np.testing.assert_array_equal(r.labels.cpu().numpy(), exp.labels, err_msg="request %d" % k)
        assert r.iterations == exp.iterations

"""Continuous batching (gsl_session) against the CPU oracle: graphs that join
a resident batch between sweeps, while others are running, get exactly the
labels and sweep counts gsl_lpa (and the oracle, Alg. 3 + Alg. 2) gives them
alone; finished graphs leave and their space is reused (compaction); bad
input is rejected per graph."""
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


def _graphs():
    b = workloads.make(5, small=True)  # 64 planted graphs, 200 .. 20,000 vertices
    gs = [b.subgraph(k) for k in range(b.num_graphs)]
    gs.append(graphgen.cliques([4, 5, 6], perm=np.random.default_rng(3).permutation(15)))
    gs.append(graphgen.from_undirected(2, [(0, 1)]))        # K2: runs to the cap
    gs.append(graphgen.from_entries(9, [], []))             # isolated vertices only
    return gs


def _run(gsl, sess, order, graphs, admit_every=1, sweeps=1):
    """Admits graphs in `order`, a few before every step, until all finished.
    Returns {index: (labels, sweeps)}."""
    pending = list(order)
    tickets, res = {}, {}
    outs = {}
    steps = 0
    while pending or tickets:
        batch = pending[:admit_every]
        if batch:
            got = sess.add([to_device(graphs[i]) for i in batch])
            for i, (t, st, lab) in zip(batch, got):
                if st == gsl.GSL_EAGAIN:
                    break
                assert st == gsl.GSL_OK, (i, st)
                pending.remove(i)
                if t < 0:
                    res[i] = (lab.cpu().numpy(), 0)
                else:
                    tickets[t] = i
                    outs[i] = lab
        if tickets:
            for t, it in sess.step(sweeps):
                i = tickets.pop(t)
                res[i] = (outs[i].cpu().numpy(), it)
            steps += 1
        assert steps < 10_000
    return res


def test_graphs_joining_a_running_batch_match_the_oracle(gsl):
    graphs = _graphs()
    refs = [oracle.lpa(g, 20, 0.05) for g in graphs]
    rng = np.random.default_rng(7)
    for admit_every, sweeps in ((1, 1), (5, 2), (len(graphs), 3)):
        order = list(rng.permutation(len(graphs)))
        with gsl.Session(400_000, 8_000_000, 128) as sess:
            res = _run(gsl, sess, order, graphs, admit_every, sweeps)
        for i, g in enumerate(graphs):
            lab, it = res[i]
            np.testing.assert_array_equal(lab, refs[i].labels, err_msg="graph %d (%d, %d)" % (i, admit_every, sweeps))
            if g.n:
                assert it == refs[i].iterations, (i, it, refs[i].iterations)


def test_alone_and_in_the_mix_are_identical(gsl):
    """A graph run alone in a session and the same graph admitted into a
    session that is mid-way through other graphs' sweeps."""
    graphs = _graphs()
    target = 10
    with gsl.Session(400_000, 8_000_000, 128) as sess:
        alone = _run(gsl, sess, [target], graphs)[target]
    with gsl.Session(400_000, 8_000_000, 128) as sess:
        others = [i for i in range(20) if i != target]
        got = sess.add([to_device(graphs[i]) for i in others])
        live = {t: i for i, (t, st, _) in zip(others, got) if t >= 0}
        sess.step(2)                                   # the others are running
        (t, st, lab), = sess.add([to_device(graphs[target])])
        assert st == gsl.GSL_OK and t >= 0
        done = {}
        while t not in done:
            for tt, it in sess.step(1):
                done[tt] = it
        mixed = (lab.cpu().numpy(), done[t])
    np.testing.assert_array_equal(alone[0], mixed[0])
    assert alone[1] == mixed[1]
    np.testing.assert_array_equal(mixed[0], oracle.lpa(graphs[target]).labels)


def test_full_session_asks_to_retry_and_compacts(gsl):
    """Capacity for about three graphs at once: later graphs get EAGAIN until
    finished ones leave, and their space is reused after compaction."""
    graphs = [workloads.make(1)] * 8            # 10,000 vertices, 118,942 entries each
    ref = oracle.lpa(graphs[0])
    cap_v, cap_e = 31_000, 400_000
    with gsl.Session(cap_v, cap_e, 16) as sess:
        saw_again = False
        pending, tickets, outs, res = list(range(len(graphs))), {}, {}, {}
        while pending or tickets:
            got = sess.add([to_device(graphs[i]) for i in pending])
            for i, (t, st, lab) in zip(list(pending), got):
                if st == gsl.GSL_EAGAIN:
                    saw_again = True
                    break
                assert st == gsl.GSL_OK
                pending.remove(i)
                tickets[t] = i
                outs[i] = lab
            info = sess.info()
            assert info["live_vertices"] <= cap_v and info["live_entries"] <= cap_e
            for t, it in sess.step(1):
                res[tickets.pop(t)] = it
        assert saw_again
    # every graph finished with the oracle's labels and sweep count
    for i in range(len(graphs)):
        np.testing.assert_array_equal(outs[i].cpu().numpy(), ref.labels)
        assert res[i] == ref.iterations


def test_bad_graphs_are_rejected_alone(gsl):
    good = workloads.make(1)
    bad_cols = graphgen.from_entries(3, [0, 1], [1, 7])       # entry outside [0, n)
    w = graphgen.from_undirected(4, [(0, 1), (2, 3)], [2, 3])
    with gsl.Session(100_000, 1_000_000, 8) as sess:
        got = sess.add([to_device(good), to_device(bad_cols), to_device(w)])
        assert [st for _, st, _ in got] == [gsl.GSL_OK, gsl.GSL_EINVAL, gsl.GSL_EINVAL]  # unweighted session
        t, _, lab = got[0]
        done = {}
        while t not in done:
            done.update(dict(sess.step(4)))
        np.testing.assert_array_equal(lab.cpu().numpy(), oracle.lpa(good).labels)
    with gsl.Session(100_000, 1_000_000, 8, weighted=True) as sess:
        (t, st, lab), = sess.add([to_device(w)])
        assert st == gsl.GSL_OK
        done = {}
        while t not in done:
            done.update(dict(sess.step(4)))
        np.testing.assert_array_equal(lab.cpu().numpy(), oracle.lpa(w).labels)


def test_session_capacity_and_bytes(gsl):
    b = gsl.Session.device_bytes(1 << 20, 1 << 24, 256)
    assert b > (1 << 24) * 4 * 2
    with gsl.Session(1 << 20, 1 << 24, 256) as sess:
        info = sess.info()
        assert info["device_bytes"] == b and info["live_graphs"] == 0
    with pytest.raises(gsl.GslError):
        gsl.Session(0, 10, 1)


def test_hub_graphs_in_a_session(gsl):
    """Graphs with hub rows (degree above 4,096) joining a running session:
    the hub tier's chunk sums, staging and merge run over the arena's hubs --
    with the default limits, and with 1 MiB staging batches and 8 merge claims
    per pass, so the several-batch and sub-pass branches run too -- and every
    graph still gets the oracle's labels and sweep count."""
    graphs = [graphgen.rmat(16, 32, 7), graphgen.rmat(14, 32, 1), graphgen.rmat(15, 16, 4)]
    b = workloads.make(5, small=True)
    graphs += [b.subgraph(k) for k in range(6)]
    assert sum(int((np.diff(g.offsets) > 4096).sum()) for g in graphs) >= 10
    refs = [oracle.lpa(g, 20, 0.05) for g in graphs]
    order = list(np.random.default_rng(5).permutation(len(graphs)))
    for limits in ((0, 0), (1 << 20, 8)):
        gsl.gsl_set_hub_limits(*limits)
        try:
            with gsl.Session(400_000, 12_000_000, 16) as sess:
                res = _run(gsl, sess, order, graphs, admit_every=1, sweeps=2)
        finally:
            gsl.gsl_set_hub_limits(0, 0)
        for i, g in enumerate(graphs):
            lab, it = res[i]
            np.testing.assert_array_equal(lab, refs[i].labels, err_msg="graph %d limits %s" % (i, limits))
            assert it == refs[i].iterations, (i, limits)


def test_descriptors_rejected_on_the_host(gsl):
    """A descriptor with NULL offsets, or a negative vertex count, is rejected
    (GSL_EINVAL) before anything on the device reads it; the good graph of
    the same call runs as usual."""
    import ctypes
    lib = gsl.load()
    good = workloads.make(1)
    off, cols, _ = to_device(good)
    out = torch.empty(good.n, dtype=torch.int32, device="cuda")
    spare = torch.empty(8, dtype=torch.int32, device="cuda")
    tab = (gsl._Graph * 3)()
    tab[0].offsets, tab[0].cols, tab[0].labels_out, tab[0].n = None, None, spare.data_ptr(), 5
    tab[1].offsets, tab[1].cols, tab[1].labels_out, tab[1].n = off.data_ptr(), cols.data_ptr(), out.data_ptr(), good.n
    tab[2].offsets, tab[2].cols, tab[2].labels_out, tab[2].n = off.data_ptr(), cols.data_ptr(), spare.data_ptr(), -3
    tickets = (ctypes.c_int64 * 3)()
    status = (ctypes.c_int32 * 3)()
    with gsl.Session(100_000, 1_000_000, 8) as sess:
        sess.stream.wait_stream(torch.cuda.current_stream())
        assert lib.gsl_session_add(sess._h, 3, tab, tickets, status) == gsl.GSL_OK
        assert list(status) == [gsl.GSL_EINVAL, gsl.GSL_OK, gsl.GSL_EINVAL]
        assert tickets[0] == -1 and tickets[2] == -1 and tickets[1] >= 0
        done = {}
        while tickets[1] not in done:
            done.update(dict(sess.step(4)))
        np.testing.assert_array_equal(out.cpu().numpy(), oracle.lpa(good).labels)

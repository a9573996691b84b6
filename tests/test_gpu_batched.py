"""GPU parity of the batched entry points against the CPU oracle run on each
graph alone.

A batch must give every graph exactly what gsl_lpa gives it alone (Alg. 3 with
its own convergence test dN_g / n_g <= tau, then Alg. 2): labels, and the
sweep count of each graph, bit-exact.  Covered: the concatenated-CSR form
(gsl_lpa_batched), separate graphs (gsl_lpa_graphs) on the shared scratch and
on contexts, contexts used from two threads at once, and the cached loop
graph being rebuilt when the batch changes.
"""
import threading

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


def concat(graphs, weighted=False):
    """Concatenated CSR of separate graphs: global entry offsets, local cols."""
    vb = np.zeros(len(graphs) + 1, dtype=np.int64)
    eb = np.zeros(len(graphs) + 1, dtype=np.int64)
    for k, g in enumerate(graphs):
        vb[k + 1] = vb[k] + g.n
        eb[k + 1] = eb[k] + g.nnz
    off = np.zeros(int(vb[-1]) + 1, dtype=np.int64)
    for k, g in enumerate(graphs):
        off[vb[k]:vb[k + 1]] = g.offsets[:-1] + eb[k]
    off[-1] = eb[-1]
    cols = np.concatenate([g.cols for g in graphs] + [np.zeros(0, np.int32)]).astype(np.int32)
    w = None
    if weighted:
        w = np.concatenate([g.weights if g.weights is not None else np.ones(g.nnz, np.uint32)
                            for g in graphs] + [np.zeros(0, np.uint32)]).astype(np.uint32)
    return graphgen.Graph(off, cols, w, vtx_base=vb, edge_base=eb, name="concat")


def expected(graphs, max_iters, tol, split=True):
    return [oracle.lpa(g, max_iters, tol, split=split) for g in graphs]


def check(labels, iters, graphs, exp, tag):
    assert len(iters) == len(graphs)
    for k, (g, r) in enumerate(zip(graphs, exp)):
        lab = labels[k]
        assert iters[k] == r.iterations, (tag, k, iters[k], r.iterations)
        np.testing.assert_array_equal(lab, r.labels, err_msg="%s graph %d (n=%d)" % (tag, k, g.n))


def run_concat(gsl, b, max_iters=20, tol=0.05, split=True, prune=True):
    off, cols, w = to_device(b)
    vb = torch.from_numpy(b.vtx_base).cuda()
    eb = torch.from_numpy(b.edge_base).cuda()
    lab, iters, st = gsl.gsl_lpa_batched(vb, eb, off, cols, w, max_iters, tol, prune=prune, split=split)
    lab = lab.cpu().numpy()
    out = [lab[b.vtx_base[k]:b.vtx_base[k + 1]] for k in range(b.num_graphs)]
    return out, iters.cpu().tolist(), st


def run_graphs(gsl, graphs, max_iters=20, tol=0.05, split=True, ctx=None):
    dev = [to_device(g) for g in graphs]
    outs, iters, st = gsl.gsl_lpa_graphs([(o, c, w) for o, c, w in dev], max_iters, tol, split=split, ctx=ctx)
    return [o.cpu().numpy() for o in outs], iters, st


def mixed_graphs(seed):
    """Edge cases in one batch: empty, isolated-only, one vertex, K2, a star,
    a self-loop-only graph, weighted multigraphs, cliques and planted graphs
    of very different sizes."""
    rng = np.random.default_rng(seed)
    gs = [graphgen.from_entries(0, [], []), graphgen.from_entries(5, [], []),
          graphgen.from_entries(1, [], []), graphgen.from_undirected(2, [(0, 1)]),
          graphgen.from_undirected(9, [(0, j) for j in range(1, 9)]),
          graphgen.from_undirected(3, [(1, 1)]),
          graphgen.cliques([3, 4, 5], perm=rng.permutation(12))]
    for t in range(6):
        n = int(rng.integers(2, 60))
        m = int(rng.integers(0, 4 * n))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        gs.append(graphgen.from_undirected(n, edges, rng.integers(0, 6, size=m)))
    for t, n in enumerate((300, 3000, 20000)):
        gs.append(graphgen.planted(n, max(2, n // 100), 0.08, n, 100 + t))
    order = rng.permutation(len(gs))
    return [gs[i] for i in order]


def test_concat_matches_oracle_per_graph(gsl):
    b = workloads.make(5, small=True)
    graphs = [b.subgraph(k) for k in range(b.num_graphs)]
    say("batch: %d graphs, N=%d, nnz=%d" % (b.num_graphs, b.n, b.nnz))
    for split in (True, False):
        exp = expected(graphs, workloads.MAX_ITERS, workloads.TOLERANCE, split)
        labels, iters, st = run_concat(gsl, b, workloads.MAX_ITERS, workloads.TOLERANCE, split=split)
        check(labels, iters, graphs, exp, "concat split=%s" % split)
        assert st["iterations"] == max(r.iterations for r in exp)


@pytest.mark.parametrize("max_iters,tol", [(20, 0.05), (20, 0.0), (3, 0.3), (1, 0.05), (0, 0.05)])
def test_mixed_edge_cases(gsl, max_iters, tol):
    graphs = mixed_graphs(7)
    weighted = any(g.weights is not None for g in graphs)
    b = concat(graphs, weighted=weighted)
    exp = expected(graphs, max_iters, tol)
    labels, iters, _ = run_concat(gsl, b, max_iters, tol)
    check(labels, iters, graphs, exp, "concat mixed")
    labels, iters, _ = run_graphs(gsl, graphs, max_iters, tol)
    check(labels, iters, graphs, exp, "graphs mixed")


def test_pruning_off_same_result(gsl):
    graphs = mixed_graphs(9)
    b = concat(graphs, weighted=True)
    a, ia, _ = run_concat(gsl, b, prune=True)
    c, ic, _ = run_concat(gsl, b, prune=False)
    assert ia == ic
    for x, y in zip(a, c):
        np.testing.assert_array_equal(x, y)


def test_batched_equals_alone(gsl):
    graphs = mixed_graphs(11)
    labels, iters, _ = run_graphs(gsl, graphs)
    for k, g in enumerate(graphs):
        if g.n == 0:
            assert iters[k] == 0
            continue
        off, cols, w = to_device(g)
        lab, st = gsl.gsl_lpa_ex(off, cols, w, 20, 0.05)
        np.testing.assert_array_equal(labels[k], lab.cpu().numpy())
        assert iters[k] == st["iterations"]


def test_cached_loop_graph_follows_the_batch(gsl):
    ga = mixed_graphs(13)
    gb = mixed_graphs(14)
    ea, eb = expected(ga, 20, 0.05), expected(gb, 20, 0.05)
    for graphs, exp in ((ga, ea), (gb, eb), (ga, ea)):
        labels, iters, _ = run_graphs(gsl, graphs)
        check(labels, iters, graphs, exp, "cache")


def test_contexts_from_two_threads(gsl):
    sets = [mixed_graphs(20 + k) for k in range(4)]
    exps = [expected(g, 20, 0.05) for g in sets]
    results = [None] * len(sets)
    errors = []
    ctxs = [gsl.Context(), gsl.Context()]

    def work(slot):
        try:
            for k in range(slot, len(sets), 2):
                results[k] = run_graphs(gsl, sets[k], ctx=ctxs[slot])
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=work, args=(s,)) for s in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for c in ctxs:
        c.close()
    assert not errors, errors
    for k in range(len(sets)):
        labels, iters, _ = results[k]
        check(labels, iters, sets[k], exps[k], "context set %d" % k)


def test_bad_bases_are_rejected(gsl):
    graphs = mixed_graphs(3)
    b = concat(graphs)
    off, cols, w = to_device(b)
    vb = b.vtx_base.copy()
    k = next(i for i in range(1, b.num_graphs) if vb[i + 1] - vb[i] >= 2)
    vb[k] = vb[k + 1] + 1  # vtx_base decreases at k + 1
    with pytest.raises(gsl.GslError) as e:
        gsl.gsl_lpa_batched(torch.from_numpy(vb).cuda(), torch.from_numpy(b.edge_base).cuda(), off, cols, w)
    assert e.value.code == gsl.GSL_EINVAL
    eb = b.edge_base.copy()
    eb[-1] += 1  # does not end at offsets[N]
    with pytest.raises(gsl.GslError) as e:
        gsl.gsl_lpa_batched(torch.from_numpy(b.vtx_base).cuda(), torch.from_numpy(eb).cuda(), off, cols, w)
    assert e.value.code == gsl.GSL_EINVAL


def test_overflow_in_one_graph_is_reported(gsl):
    graphs = [graphgen.planted(200, 4, 0.1, 200, 1),
              graphgen.from_undirected(3, [(0, 1), (0, 2)], [1 << 31, 1 << 31])]
    with pytest.raises(gsl.GslError) as e:
        run_graphs(gsl, graphs)
    assert e.value.code == gsl.GSL_EOVERFLOW


def test_malformed_graph_fails_alone(gsl):
    graphs = mixed_graphs(5)
    exp = expected(graphs, 20, 0.05)
    dev = [list(to_device(g)) for g in graphs]
    big = max(range(len(graphs)), key=lambda k: graphs[k].nnz)
    # graph `big`: one column out of range; the next non-empty graph: decreasing offsets
    bad_cols = dev[big][1].clone()
    bad_cols[bad_cols.numel() // 2] = graphs[big].n + 5
    dev[big][1] = bad_cols
    other = next(k for k in range(len(graphs)) if k != big and graphs[k].n >= 3 and graphs[k].nnz > 0)
    bad_off = dev[other][0].clone()
    a, b = int(bad_off[1]), int(bad_off[2])
    bad_off[1], bad_off[2] = b + 1, a  # offsets[1] > offsets[2]
    dev[other][0] = bad_off
    sentinel = [torch.full((g.n,), -7, dtype=torch.int32, device="cuda") for g in graphs]
    outs, iters, _, status = gsl.gsl_lpa_graphs([(o, c, w, s) for (o, c, w), s in zip(dev, sentinel)],
                                                return_status=True)
    for k, g in enumerate(graphs):
        lab = outs[k].cpu().numpy()
        if k in (big, other):
            assert status[k] == gsl.GSL_EINVAL, k
            assert (lab == -7).all(), k
            assert iters[k] == 0
        else:
            assert status[k] == gsl.GSL_OK, k
            assert iters[k] == exp[k].iterations
            np.testing.assert_array_equal(lab, exp[k].labels)
    with pytest.raises(gsl.GslError) as e:
        gsl.gsl_lpa_graphs([(o, c, w) for o, c, w in dev])
    assert e.value.code == gsl.GSL_EINVAL
    with pytest.raises(gsl.GslError):
        gsl.gsl_check_graph(dev[big][0], dev[big][1])
    with pytest.raises(gsl.GslError):
        gsl.gsl_check_graph(dev[other][0], dev[other][1])
    gsl.gsl_check_graph(*to_device(graphs[big])[:2])


def test_full_batch_matches_oracle_hash(gsl):
    """The whole batch of 4,096 graphs (2.4B entries) in one call against the
    oracle's per-graph results (hash of the labels in graph order, sweep count
    of every graph)."""
    import json
    import os
    from tests.gpu_util import graph_hash, labels_hash
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "workloads.json")
    with open(path) as f:
        gold = json.load(f).get("5")
    if gold is None:
        pytest.skip("batched workload not in the golden file")
    b = workloads.make(5)
    assert b.n == gold["n"] and b.nnz == gold["nnz"] and b.num_graphs == gold["graphs"]
    assert graph_hash(b) == gold["graph_xxh128"]
    say("batch: %d graphs, N=%d, nnz=%d" % (b.num_graphs, b.n, b.nnz))
    # the default tiers, and the table the autotuner picks for this batch
    # (a thread per vertex up to degree 64: the benchmark's tiers)
    tuned = [(32, 16), (64, 18), (128, 8), (512, 9), (1024, 17), (2048, 11), (4096, 13)]
    try:
        for tiers in (None, tuned):
            gsl.gsl_set_tiers(tiers)
            labels, iters, _ = run_concat(gsl, b, gold["max_iters"], gold["tolerance"])
            assert iters == gold["iterations"], tiers
            assert labels_hash(np.concatenate(labels)) == gold["labels_xxh128"], tiers
    finally:
        gsl.gsl_set_tiers(None)

"""Pins of the CPU oracle against things other than itself.

* brute force on tiny graphs (every simple graph with up to 6 vertices; random
  multigraphs with duplicates, self loops and zero weights),
* closed forms (disjoint cliques, K2 and star oscillation, modularity of
  cliques / one community / singletons),
* invariants (pruning exactness, fixed point, split idempotence, no
  disconnected community after the split),
* three independent split routines (Alg. 2 BFS, Alg. 1 LP / LPP, union-find).

Paper references: Alg. 3 (lpa, lpaMove, scanCommunities) and Eq. 2 for the
sweep; Alg. 2 and Alg. 1 for the split; Eq. 1 for modularity; Alg. 4 for the
disconnected-community check; Sec. 3.2 for the modularity range.
"""
import numpy as np
import pytest

import graphgen
import oracle
from tests import brute


def _csr_from_dense(W, X):
    n = W.shape[0]
    r, c = np.nonzero(X)
    return graphgen.from_entries(n, r, c, W[r, c].astype(np.uint32))


def _check_batch(Wb, Xb, max_iters, tol, weighted=True):
    Lb, itb, dns, hist = brute.lpa(Wb, Xb, max_iters, tol)
    Sb = brute.split(Xb, Lb)
    for b in range(Wb.shape[0]):
        g = _csr_from_dense(Wb[b], Xb[b])
        if not weighted:
            g.weights = None
        for prune in (True, False):
            r = oracle.lpa(g, max_iters, tol, prune=prune, split=False, history=True)
            assert r.iterations == itb[b], (b, prune)
            for t in range(r.iterations):
                assert r.dn[t] == dns[t][b]
                np.testing.assert_array_equal(r.history[t], hist[t][b])
            np.testing.assert_array_equal(r.labels, Lb[b])
        full = oracle.lpa(g, max_iters, tol)
        np.testing.assert_array_equal(full.labels, Sb[b])


@pytest.mark.parametrize("n,tol,max_iters", [(1, 0.05, 20), (2, 0.05, 20), (3, 0.0, 20),
                                             (4, 0.25, 20), (5, 0.2, 20), (5, 0.05, 3)])
def test_exhaustive_unit_weights_small(n, tol, max_iters):
    A = brute.all_graphs(n)
    _check_batch(A.astype(np.int64), A, max_iters, tol, weighted=False)


def test_exhaustive_unit_weights_n6():
    # 32,768 graphs; tol = 1/6 sits exactly on the dN/N boundary for dN = 1.
    A = brute.all_graphs(6)
    _check_batch(A.astype(np.int64), A, 20, 1 / 6, weighted=False)


def test_exhaustive_random_weights_n5():
    A = brute.all_graphs(5)
    rng = np.random.default_rng(11)
    W = rng.integers(1, 5, size=A.shape)
    W = np.triu(W, 1)
    W = W + np.transpose(W, (0, 2, 1))
    W = np.where(A, W, 0)
    _check_batch(W, A, 20, 0.2)


def test_random_multigraphs_with_self_loops_duplicates_zero_weights():
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.integers(1, 13))
        m = int(rng.integers(0, 3 * n + 1))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        ws = rng.integers(0, 4, size=m)
        g = graphgen.from_undirected(n, edges, ws)
        W, X = brute.dense_from_graph(g)
        tol = float(rng.choice([0.0, 0.05, 0.25]))
        iters = int(rng.choice([1, 2, 20]))
        _, itb, dns, hist = brute.lpa(W[None], X[None], iters, tol)
        r = oracle.lpa(g, iters, tol, split=False, history=True)
        assert r.iterations == itb[0], trial
        for t in range(r.iterations):
            assert r.dn[t] == dns[t][0]
            np.testing.assert_array_equal(r.history[t], hist[t][0])
        rf = oracle.lpa(g, iters, tol)
        np.testing.assert_array_equal(rf.labels, brute.split(X[None], r.labels[None].astype(np.int64))[0])


def test_tiny_planted_graphs_brute_force():
    for seed in range(40):
        n = 10 + seed % 31
        g = graphgen.planted(n, max(1, n // 8), 0.5, n // 2, 1000 + seed, wmin=1, wmax=(seed % 3) * 4)
        W, X = brute.dense_from_graph(g)
        L, it, dns, _ = brute.lpa(W[None], X[None], 20, 0.05)
        r = oracle.lpa(g, 20, 0.05, split=False)
        assert r.iterations == it[0]
        np.testing.assert_array_equal(r.labels, L[0])
        np.testing.assert_array_equal(oracle.lpa(g).labels, brute.split(X[None], L)[0])


@pytest.mark.parametrize("sizes,tol", [([3, 4, 5, 6], 0.05), ([3] * 10, 0.05), ([3] * 10, 0.4),
                                       ([7, 3, 9], 0.2)])
def test_disjoint_cliques_closed_form(sizes, tol):
    # Sweep 0 changes every vertex, sweep 1 only each clique's smallest id,
    # sweep 2 nothing; the result is the smallest id of each clique.
    N = sum(sizes)
    rng = np.random.default_rng(len(sizes))
    perm = rng.permutation(N)
    g = graphgen.cliques(sizes, perm)
    r = oracle.lpa(g, 20, tol)
    k = len(sizes)
    expect_iters = 2 if k / N <= tol else 3
    assert r.iterations == expect_iters
    assert list(r.dn[:2]) == [N, k]
    if expect_iters == 3:
        assert r.dn[2] == 0
    base = 0
    for s in sizes:
        ids = perm[base:base + s]
        assert (r.labels[ids] == ids.min()).all()
        base += s


def test_k2_oscillates_until_cap():
    g = graphgen.from_undirected(2, [(0, 1)])
    r = oracle.lpa(g, 20, 0.05, split=False)
    assert r.iterations == 20 and list(r.dn) == [2] * 20
    assert list(r.labels) == [0, 1]
    r = oracle.lpa(g, 7, 0.05, split=False)
    assert list(r.labels) == [1, 0]
    # Split of the swapped labels: two singleton communities keep their ids.
    assert list(oracle.lpa(g, 7, 0.05).labels) == [0, 1]


@pytest.mark.parametrize("k", [2, 3, 10])
def test_star_oscillation_and_split(k):
    edges = [(0, j) for j in range(1, k + 1)]
    g = graphgen.from_undirected(k + 1, edges)
    r = oracle.lpa(g, 20, 0.05, split=False)
    assert r.iterations == 20 and (r.dn == k + 1).all()
    assert list(r.labels) == [0] + [1] * k
    # Leaves share label 1 but only touch the centre: every leaf is its own piece.
    assert list(oracle.lpa(g, 20, 0.05).labels) == list(range(k + 1))
    _, cnt = oracle.disconnected(g, r.labels)
    assert cnt == 1


@pytest.mark.parametrize("idx", [1, 2, 3])
def test_pruning_is_exact_on_workloads(idx):
    g = __import__("graphgen.workloads", fromlist=["make"]).make(idx, small=True)
    a = oracle.lpa(g, 20, 0.05, prune=True)
    b = oracle.lpa(g, 20, 0.05, prune=False)
    np.testing.assert_array_equal(a.labels, b.labels)
    np.testing.assert_array_equal(a.dn, b.dn)
    assert (a.processed <= b.processed).all()


def test_fixed_point_when_converged_to_zero():
    g = graphgen.cliques([4, 5, 6, 3])
    r = oracle.lpa(g, 20, 0.0, split=False)
    assert r.dn[-1] == 0
    W, X = brute.dense_from_graph(g)
    best = brute.best_labels(W[None], X[None], r.labels[None].astype(np.int64))[0]
    np.testing.assert_array_equal(best, r.labels)


def _union_find_split(g, C):
    n = g.n
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u in range(n):
        for e in range(g.offsets[u], g.offsets[u + 1]):
            v = int(g.cols[e])
            if C[u] == C[v]:
                a, b = find(u), find(v)
                if a != b:
                    parent[max(a, b)] = min(a, b)
    return np.array([find(i) for i in range(n)], dtype=np.int32)


def test_split_routines_agree():
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(1, 60))
        g = graphgen.planted(n, max(1, n // 6), 0.3, n, 77 + trial)
        C = rng.integers(0, max(1, n // 4), size=n).astype(np.int32)
        a = oracle.split_bfs(g, C)
        b, _ = oracle.split_lp(g, C, prune=False)
        c, _ = oracle.split_lp(g, C, prune=True)
        d = _union_find_split(g, C)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(a, c)
        np.testing.assert_array_equal(a, d)
        if n <= 40:
            W, X = brute.dense_from_graph(g)
            np.testing.assert_array_equal(a, brute.split(X[None], C[None].astype(np.int64))[0])
        assert (a <= np.arange(n)).all()
        np.testing.assert_array_equal(a[a], a)
        assert oracle.disconnected(g, a)[1] == 0


def test_disconnected_matches_component_count():
    rng = np.random.default_rng(9)
    for trial in range(40):
        n = int(rng.integers(1, 30))
        g = graphgen.planted(n, max(1, n // 5), 0.25, n // 2, 500 + trial)
        C = rng.integers(0, max(1, n // 3), size=n).astype(np.int32)
        D, cnt = oracle.disconnected(g, C)
        W, X = brute.dense_from_graph(g)
        comps = brute.components_per_label(X, C.astype(np.int64))
        expect = {c for c, k in comps.items() if k > 1}
        assert set(np.nonzero(D)[0].tolist()) == expect
        assert cnt == len(expect)


def test_workload_outputs_have_no_disconnected_communities():
    from graphgen.workloads import make
    for idx in (1, 2, 3):
        g = make(idx, small=True)
        raw = oracle.lpa(g, 20, 0.05, split=False).labels
        out = oracle.lpa(g, 20, 0.05).labels
        assert oracle.disconnected(g, out)[1] == 0
        np.testing.assert_array_equal(out, oracle.split_bfs(g, raw))


# ---------------------------------------------------------------- modularity

@pytest.mark.parametrize("k,s", [(2, 3), (5, 4), (10, 10)])
def test_modularity_equal_cliques(k, s):
    g = graphgen.cliques([s] * k)
    lab = np.repeat(np.arange(k) * s, s).astype(np.int32)
    assert abs(oracle.modularity(g, lab) - (1 - 1 / k)) < 1e-15


def test_modularity_general_cliques_one_community_singletons():
    sizes = [3, 5, 8, 13]
    g = graphgen.cliques(sizes)
    lab = np.concatenate([np.full(s, sum(sizes[:t])) for t, s in enumerate(sizes)]).astype(np.int32)
    two_m = sum(s * (s - 1) for s in sizes)
    expect = 1 - sum((s * (s - 1) / two_m) ** 2 for s in sizes)
    assert abs(oracle.modularity(g, lab) - expect) < 1e-15
    n = g.n
    assert oracle.modularity(g, np.zeros(n, dtype=np.int32)) == 0.0
    K = np.diff(g.offsets).astype(np.float64)
    assert abs(oracle.modularity(g, np.arange(n, dtype=np.int32)) + ((K / two_m) ** 2).sum()) < 1e-15


def test_modularity_brute_force_pairs_and_range():
    rng = np.random.default_rng(21)
    for trial in range(200):
        n = int(rng.integers(1, 25))
        g = graphgen.planted(n, max(1, n // 4), 0.4, n, 900 + trial, wmin=1, wmax=int(rng.integers(0, 6)))
        lab = rng.integers(0, n, size=n).astype(np.int32)
        if trial % 3 == 0:
            lab = oracle.lpa(g).labels
        W, _ = brute.dense_from_graph(g)
        q = oracle.modularity(g, lab)
        assert abs(q - brute.modularity_pairs(W, lab.astype(np.int64))) < 1e-12
        assert -0.5 - 1e-12 <= q <= 1 + 1e-12


def test_modularity_integer_parts():
    g = graphgen.planted(300, 6, 0.2, 300, 4, wmin=1, wmax=9)
    lab = oracle.lpa(g).labels
    q, (two_m, I, S2) = oracle.modularity(g, lab, parts=True)
    assert two_m == int(g.weights.astype(np.int64).sum())
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets))
    w = g.weights.astype(np.int64)
    assert I == int(w[lab[rows] == lab[g.cols]].sum())
    Sig = np.bincount(lab[rows], weights=w, minlength=g.n).astype(np.int64)
    assert S2 == sum(int(x) * int(x) for x in Sig)


def test_oracle_rejects_bad_input():
    g = graphgen.from_entries(3, [0, 1], [1, 5])
    with pytest.raises(ValueError):
        oracle.lpa(g)
    g = graphgen.from_undirected(3, [(0, 1)])
    with pytest.raises(ValueError):
        oracle.split_bfs(g, np.array([0, 1, 3], dtype=np.int32))


# ---- fp32 weights summed in fp64 (the paper's precision) ----

def test_f32_integer_weights_reduce_to_the_integer_oracle():
    rng = np.random.default_rng(41)
    for trial in range(40):
        n = int(rng.integers(2, 300))
        g = graphgen.planted(n, max(1, n // 20), 0.2, n, 100 + trial, wmin=1, wmax=50)
        a = oracle.lpa(g, 20, 0.05)
        b = oracle.lpa_f32(g, g.weights.astype(np.float32), 20, 0.05)
        assert a.iterations == b.iterations
        np.testing.assert_array_equal(a.labels, b.labels)
        np.testing.assert_array_equal(a.dn, b.dn)


def test_f32_brute_force_dyadic_weights():
    """Every graph on 5 vertices with random dyadic weights k/64 (every partial
    sum exact in fp64, so summation order cannot matter) against the dense
    fp64 brute force, sweep by sweep."""
    rng = np.random.default_rng(42)
    A = brute.all_graphs(5)
    Wd = rng.integers(1, 200, size=A.shape) / 64.0
    Wd = np.triu(Wd, 1)
    Wd = Wd + np.transpose(Wd, (0, 2, 1))
    W = np.where(A, Wd, 0.0)
    L, iters, dns, _ = brute.lpa(W, A, 20, 0.2)
    for b in range(A.shape[0]):
        r, c = np.nonzero(A[b])
        g = graphgen.from_entries(5, r, c)
        w = W[b][r, c].astype(np.float32)
        res = oracle.lpa_f32(g, w, 20, 0.2, split=False)
        assert res.iterations == iters[b], b
        np.testing.assert_array_equal(res.labels, L[b], err_msg="graph %d" % b)


def test_f32_sums_are_fp64_not_fp32():
    """Row of vertex 0: label 2 twice (1.0 and 2^-25), label 1 once (1.0).  In
    fp64 label 2 weighs 1 + 2^-25 and wins; summed in fp32 it would tie at 1.0
    and the smaller label 1 would win."""
    g = graphgen.from_entries(3, [0, 0, 0, 1, 2, 2], [2, 2, 1, 0, 0, 0])
    w = np.array([1.0, 2.0 ** -25, 1.0, 1.0, 1.0, 2.0 ** -25], dtype=np.float32)
    r = oracle.lpa_f32(g, w, 1, 0.0, split=False)
    assert r.labels[0] == 2
    assert np.float32(1.0) + np.float32(2.0 ** -25) == np.float32(1.0)  # the fp32 tie it avoids


def test_f32_rejects_negative_and_nan_weights():
    g = graphgen.from_undirected(3, [(0, 1), (1, 2)])
    for bad in (-1.0, float("nan"), float("inf")):
        w = np.ones(g.nnz, dtype=np.float32)
        w[1] = bad
        with pytest.raises(ValueError):
            oracle.lpa_f32(g, w)

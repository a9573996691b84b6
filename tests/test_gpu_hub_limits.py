"""GPU tests of the hub tier's rarely taken branches and of the loop-graph
cache, each compared element by element with the CPU oracle (Alg. 3 /
Eq. 2 sweeps, Alg. 2 split).

  - hub rows summed over several staging batches (every batch after the
    first starts at a hub k0 > 0) and partitions merged in hashed
    sub-passes, forced on small graphs with gsl_set_hub_limits;
  - sweeps of thousands of hub batches, which the loop graph holds one
    sweep at a time or not at all;
  - the cached loop graph is rebuilt when only the hub chunk totals change
    (two graphs with equal n, nnz, tier counts and hub count, at the same
    device addresses);
  - a row whose weights sum to 2^32 or more in an LDS or hub tier, where a
    packed (label, sum) slot can carry into the label: the call fails with
    GSL_EOVERFLOW and no label outside [0, n) is ever written.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import graphgen  # noqa: E402
import oracle  # noqa: E402
from graphgen import workloads  # noqa: E402
from tests.gpu_util import say, to_device  # noqa: E402

pytestmark = pytest.mark.gpu

# Hubs above degree 256 (the remaining levels keep their variants).
LOW_HUB_LEVELS = [(8, 0), (16, 15), (32, 16), (64, 6), (128, 8), (256, 9), (256, 9)]


@pytest.fixture(scope="module")
def gsl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_01261_amd as m
    m.load()
    yield m
    m.gsl_set_tiers(None)
    m.gsl_set_hub_limits(0, 0)


def check(gsl, g, max_iters=20, tol=0.05, layouts=("original", "renumbered"), tag=""):
    for split in (False, True):
        r = oracle.lpa(g, max_iters, tol, split=split)
        for layout in layouts:
            off, cols, w = to_device(g)
            lab, st = gsl.gsl_lpa_ex(off, cols, w, max_iters, tol, split=split, layout=layout)
            assert st["iterations"] == r.iterations, (tag, split, layout)
            k = min(r.iterations, 64)
            assert list(st["changed"][:k]) == list(r.dn[:k]), (tag, split, layout)
            np.testing.assert_array_equal(lab.cpu().numpy(), r.labels,
                                          err_msg="%s split=%s %s" % (tag, split, layout))


def _hub_graph(seed, hub_degrees, n=40_000, weighted=False):
    """Planted background plus hubs of the given degrees (distinct random
    neighbours)."""
    rng = np.random.default_rng(seed)
    base = graphgen.planted(n, 400, 0.02, n, seed)
    rows = np.repeat(np.arange(n), np.diff(base.offsets))
    keep = rows < base.cols
    edges = set(zip(rows[keep].tolist(), base.cols[keep].tolist()))
    for k, deg in enumerate(hub_degrees):
        v = 997 * k + 13
        nb = rng.choice(n, size=deg + 10, replace=False)
        for u in [int(x) for x in nb if x != v][:deg]:
            edges.add((min(u, v), max(u, v)))
    edges = sorted(edges)
    ws = rng.integers(1, 9, size=len(edges)) if weighted else None
    return graphgen.from_undirected(n, edges, ws)


@pytest.mark.parametrize("weighted", [False, True])
def test_hub_staging_batches(gsl, weighted):
    """Staging room for two chunks: every hub (at least 3 chunks) gets a
    batch of its own, so batches 2.. start at k0 > 0."""
    g = _hub_graph(21 + weighted, [4500, 5000, 9000, 12_000, 20_000], weighted=weighted)
    say("hub graph n=%d nnz=%d maxdeg=%d" % (g.n, g.nnz, np.diff(g.offsets).max()))
    try:
        gsl.gsl_set_hub_limits(2 * 2048 * 8, 0)
        check(gsl, g, tag="staging 2 chunks")
        gsl.gsl_set_hub_limits(7 * 2048 * 8, 0)  # batches of one or two hubs
        check(gsl, g, tag="staging 7 chunks")
    finally:
        gsl.gsl_set_hub_limits(0, 0)


@pytest.mark.parametrize("cap", [8, 64, 1000])
def test_hub_merge_subpasses(gsl, cap):
    """A merge pass that accepts only `cap` distinct labels: partitions of
    sweep 0 (all labels distinct) are merged in 2, 4, ... hashed sub-passes,
    later sweeps mostly fit one pass."""
    g = _hub_graph(31, [4200, 6000, 14_000])
    try:
        gsl.gsl_set_hub_limits(0, cap)
        check(gsl, g, tag="merge cap %d" % cap)
    finally:
        gsl.gsl_set_hub_limits(0, 0)


def test_hub_limits_on_rmat_with_low_hub_bound(gsl):
    """R-MAT (small workload 4) with every row above degree 256 in the hub
    tier, tiny staging batches and a small merge cap, at once."""
    g = workloads.make(4, small=True)
    try:
        gsl.gsl_set_tiers(LOW_HUB_LEVELS)
        gsl.gsl_set_hub_limits(5 * 2048 * 8, 40)
        check(gsl, g, tag="rmat small, hubs > 256")
    finally:
        gsl.gsl_set_tiers(None)
        gsl.gsl_set_hub_limits(0, 0)


@pytest.mark.parametrize("hub_above", [256, 128])
def test_wide_hub_sweeps(gsl, hub_above):
    """One staging chunk per batch over R-MAT's 2,517 rows above degree 256
    (a sweep of about 10^4 launches: loop graphs of one sweep each) or its
    6,834 rows above 128 (about 2.7 * 10^4: no loop graph, sweeps launched
    directly)."""
    g = workloads.make(4, small=True)
    levels = LOW_HUB_LEVELS if hub_above == 256 else LOW_HUB_LEVELS[:4] + [(128, 8)] * 3
    try:
        gsl.gsl_set_tiers(levels)
        gsl.gsl_set_hub_limits(2048 * 8, 0)
        check(gsl, g, tag="rmat small, hubs > %d, one chunk per batch" % hub_above)
    finally:
        gsl.gsl_set_tiers(None)
        gsl.gsl_set_hub_limits(0, 0)


def test_hub_limits_reject_bad_values(gsl):
    for bad in ((-1, 0), (100, 0), (0, -1), (0, 4000)):
        with pytest.raises(gsl.GslError) as e:
            gsl.gsl_set_hub_limits(*bad)
        assert e.value.code == gsl.GSL_EINVAL
    gsl.gsl_set_hub_limits(0, 0)


def _three_hubs(degrees, heavy_last):
    """Hubs 0, 1, 2 with the given degrees over distinct leaves 3 .. (each
    leaf has degree 1) plus isolated vertices up to a fixed n.  The last
    neighbour of the last hub weighs 1000, so the hub's winner sits in its
    last chunk."""
    n = 3 + sum(degrees) + 100
    edges, ws = [], []
    leaf = 3
    for h, d in enumerate(degrees):
        for k in range(d):
            edges.append((h, leaf))
            ws.append(1000 if (heavy_last and h == len(degrees) - 1 and k == d - 1) else 1)
            leaf += 1
    return graphgen.from_undirected(n, edges, ws)


def test_loop_graph_rebuilt_when_hub_chunks_change(gsl):
    """Two graphs with equal n, nnz, tier counts, hub count and largest
    partition count, but 11 and 12 hub chunks, run from the same device
    buffers after a larger hub graph has grown the hub scratch: each result
    must match the oracle (a cached loop graph with the other's hub grids
    would skip or add chunks)."""
    big = _three_hubs([9000, 20_000, 30_000], False)
    b = _three_hubs([6144, 6144, 10240], True)
    c = _three_hubs([4097, 8191, 10240], True)
    assert b.n == c.n and b.nnz == c.nnz
    assert np.array_equal(np.bincount(np.diff(b.offsets) > 4096), np.bincount(np.diff(c.offsets) > 4096))
    for layout in ("original", "renumbered"):
        off_big, cols_big, w_big = to_device(big)
        gsl.gsl_lpa_ex(off_big, cols_big, w_big, 20, 0.05, layout=layout)
        off = torch.empty(b.n + 1, dtype=torch.int64, device="cuda")
        cols = torch.empty(b.nnz, dtype=torch.int32, device="cuda")
        w = torch.empty(b.nnz, dtype=torch.int32, device="cuda")
        out = torch.empty(b.n, dtype=torch.int32, device="cuda")
        for g in (b, c, b, c):
            o, cc, ww = to_device(g)
            off.copy_(o)
            cols.copy_(cc)
            w.copy_(ww)
            for split in (False, True):
                r = oracle.lpa(g, 20, 0.05, split=split)
                lab, st = gsl.gsl_lpa_ex(off, cols, w, 20, 0.05, split=split, layout=layout, out=out)
                assert st["iterations"] == r.iterations, (layout, split)
                np.testing.assert_array_equal(lab.cpu().numpy(), r.labels, err_msg="%s split=%s" % (layout, split))


def _overflow_graph(deg, n_extra=10):
    """Vertex 0 with `deg` entries: two entries to the last vertex n - 1
    weighing 2^31 each (a duplicate entry: one label summing to 2^32, which
    carries into the label half of a packed slot), the rest weight 1."""
    n = deg + n_extra
    rows, cols, ws = [], [], []
    for j in range(1, deg - 1):
        rows += [0, j]
        cols += [j, 0]
        ws += [1, 1]
    rows += [0, 0, n - 1, n - 1]
    cols += [n - 1, n - 1, 0, 0]
    ws += [1 << 31, 1 << 31, 1 << 31, 1 << 31]
    return graphgen.from_entries(n, rows, cols, ws)


@pytest.mark.parametrize("deg,levels", [(20, None), (70, None), (600, None), (5000, None),
                                        (400, LOW_HUB_LEVELS)])
def test_overflow_reported_in_every_tier(gsl, deg, levels):
    g = _overflow_graph(deg)
    try:
        gsl.gsl_set_tiers(levels)
        for layout in ("original", "renumbered"):
            for asyn in (False, True):
                off, cols, w = to_device(g)
                out = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
                with pytest.raises(gsl.GslError) as e:
                    gsl.gsl_lpa_ex(off, cols, w, 20, 0.05, layout=layout, async_sweeps=asyn, out=out)
                assert e.value.code == gsl.GSL_EOVERFLOW, (deg, layout, asyn)
                got = out.cpu().numpy()
                # whatever was written is a vertex id (or untouched)
                assert ((got == -7) | ((got >= 0) & (got < g.n))).all(), (deg, layout, asyn)
        # the library is usable afterwards
        ok = workloads.make(1)
        o, c, ww = to_device(ok)
        lab, _ = gsl.gsl_lpa_ex(o, c, ww, 20, 0.05)
        np.testing.assert_array_equal(lab.cpu().numpy(), oracle.lpa(ok).labels)
    finally:
        gsl.gsl_set_tiers(None)

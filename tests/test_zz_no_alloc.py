"""gsl_lpa_noalloc (no device allocation, static scratch) against gsl_lpa
through the C ABI: identical labels on consecutive calls, the later ones on
smaller graphs (the static array keeps the previous call's contents), and
the size limits rejected before any device work."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import graphgen  # noqa: E402
import oracle  # noqa: E402
from graphgen import workloads  # noqa: E402
from tests.gpu_util import say, to_device  # noqa: E402

pytestmark = pytest.mark.gpu

LOW_HUB_LEVELS = [(8, 0), (16, 15), (32, 16), (64, 6), (128, 8), (256, 9), (256, 9)]


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_01261_amd as m
    m.load()
    yield m
    m.gsl_set_tiers(None)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _hub_graph(seed, n, hub_degrees, weighted):
    rng = np.random.default_rng(seed)
    base = graphgen.planted(n, n // 100, 0.03, n, seed)
    rows = np.repeat(np.arange(n), np.diff(base.offsets))
    keep = rows < base.cols
    edges = set(zip(rows[keep].tolist(), base.cols[keep].tolist()))
    for k, deg in enumerate(hub_degrees):
        v = 991 * k + 5
        for u in rng.choice(n, size=deg, replace=False).tolist():
            if u != v:
                edges.add((min(u, v), max(u, v)))
    edges = sorted(edges)
    ws = rng.integers(1, 17, size=len(edges)) if weighted else None
    return graphgen.from_undirected(n, edges, ws)


def _both(lib, g, max_iters=20, tol=0.05):
    """Labels of gsl_lpa and of gsl_lpa_noalloc, both called through the C
    ABI on the same device arrays."""
    L = lib.load()
    lib._bind_stream()
    off, cols, w = to_device(g)
    n = g.n
    ref = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    got = torch.full((n,), -2, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    rc = L.gsl_lpa(_ptr(off), _ptr(cols), _ptr(w), n, max_iters, tol, _ptr(ref))
    assert rc == lib.GSL_OK, L.gsl_last_error()
    rc = L.gsl_lpa_noalloc(_ptr(off), _ptr(cols), _ptr(w), n, max_iters, tol, _ptr(got))
    assert rc == lib.GSL_OK, L.gsl_last_error()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_equals_gsl_lpa_on_calls_of_decreasing_size(lib):
    graphs = [_hub_graph(3, 60_000, [9000, 30_000], True),   # hubs, weights
              workloads.make(2, small=True),                  # R-MAT, weights
              workloads.make(1),                              # planted 10k
              graphgen.cliques([4, 5, 6])]                    # tiny
    sizes = [g.n for g in graphs]
    assert sizes == sorted(sizes, reverse=True)
    for k, g in enumerate(graphs):
        say("noalloc call %d: n=%d nnz=%d" % (k, g.n, g.nnz))
        ref, got = _both(lib, g)
        np.testing.assert_array_equal(got, ref, err_msg="call %d" % k)
        np.testing.assert_array_equal(got, oracle.lpa(g).labels, err_msg="call %d vs oracle" % k)


def test_noalloc_hub_batches_and_low_tiers(lib):
    """Many hub rows (every row above degree 256) in staging batches of the
    static area, then a smaller graph again."""
    try:
        lib.gsl_set_tiers(LOW_HUB_LEVELS)
        for g in (workloads.make(4, small=True), workloads.make(1)):
            say("noalloc low tiers: n=%d nnz=%d" % (g.n, g.nnz))
            ref, got = _both(lib, g)
            np.testing.assert_array_equal(got, ref)
    finally:
        lib.gsl_set_tiers(None)


def test_noalloc_limits_rejected(lib):
    L = lib.load()
    off = torch.zeros(4, dtype=torch.int64, device="cuda")
    cols = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.zeros(4, dtype=torch.int32, device="cuda")
    # n above the maximum, max_iters above the maximum: rejected on the host
    assert L.gsl_lpa_noalloc(_ptr(off), _ptr(cols), None, (1 << 20) + 1, 20, 0.05, _ptr(out)) == lib.GSL_EINVAL
    assert b"exceeds" in L.gsl_last_error()
    assert L.gsl_lpa_noalloc(_ptr(off), _ptr(cols), None, 3, 257, 0.05, _ptr(out)) == lib.GSL_EINVAL
    assert L.gsl_lpa_noalloc(None, None, None, 0, 20, 0.05, None) == lib.GSL_OK
    # and the entry point still works afterwards
    g = graphgen.from_undirected(3, [(0, 1), (1, 2)])
    ref, got = _both(lib, g)
    np.testing.assert_array_equal(got, ref)

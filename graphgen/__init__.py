"""Seeded synthetic CSR graphs (inputs only; no community-detection arithmetic).

Both the CPU oracle and the GPU library are fed from here.  The native part
(`graphgen.cpp`) is compiled with g++ into ``libgraphgen.so`` next to this file;
the small hand-made graphs used by tests are built in plain numpy below.

Every graph is returned as a :class:`Graph` with numpy arrays
``offsets`` (int64[n+1]), ``cols`` (int32[nnz]) and ``weights`` (uint32[nnz] or
``None`` for unit weights).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build(force: bool = True) -> str:
    """Compile libgraphgen.so (portable x86-64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _GG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("cols", ctypes.POINTER(ctypes.c_int32)),
                ("weights", ctypes.POINTER(ctypes.c_uint32)),
                ("num_graphs", ctypes.c_int64),
                ("vtx_base", ctypes.POINTER(ctypes.c_int64)),
                ("edge_base", ctypes.POINTER(ctypes.c_int64))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_GG)
        lib.gg_free.argtypes = [P]
        lib.gg_planted.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_int64,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, P]
        lib.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32,
                                ctypes.c_uint64, P]
        lib.gg_road_knn.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, P]
        lib.gg_batched_planted.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_uint64, P]
        for f in (lib.gg_planted, lib.gg_rmat, lib.gg_road_knn, lib.gg_batched_planted):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class Graph:
    """Symmetric CSR graph.  ``vtx_base``/``edge_base`` are set for batches."""

    def __init__(self, offsets, cols, weights=None, vtx_base=None, edge_base=None, name=""):
        self.offsets = offsets
        self.cols = cols
        self.weights = weights
        self.vtx_base = vtx_base
        self.edge_base = edge_base
        self.name = name

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0]) - 1

    @property
    def nnz(self) -> int:
        return int(self.cols.shape[0])

    @property
    def num_graphs(self) -> int:
        return 1 if self.vtx_base is None else int(self.vtx_base.shape[0]) - 1

    def subgraph(self, g: int) -> "Graph":
        """Graph g of a batch as a standalone CSR (local ids, copies)."""
        vb, ve = int(self.vtx_base[g]), int(self.vtx_base[g + 1])
        eb, ee = int(self.edge_base[g]), int(self.edge_base[g + 1])
        off = (self.offsets[vb:ve + 1] - eb).astype(np.int64)
        w = None if self.weights is None else self.weights[eb:ee].copy()
        return Graph(off, self.cols[eb:ee].copy(), w, name="%s[%d]" % (self.name, g))

    def unit_weights(self) -> np.ndarray:
        return np.ones(self.nnz, dtype=np.uint32)


def _wrap(st: _GG, name: str) -> Graph:
    lib = _load()
    holder = ctypes.pointer(st)
    n, nnz = st.n, st.nnz

    def arr(ptr, count, dtype):
        if not ptr or count == 0:
            return np.zeros(count, dtype=dtype)
        return np.ctypeslib.as_array(ptr, shape=(count,))

    off = arr(st.offsets, n + 1, np.int64)
    cols = arr(st.cols, nnz, np.int32)
    w = arr(st.weights, nnz, np.uint32) if st.weights else None
    vb = arr(st.vtx_base, st.num_graphs + 1, np.int64) if st.vtx_base else None
    eb = arr(st.edge_base, st.num_graphs + 1, np.int64) if st.edge_base else None
    g = Graph(off, cols, w, vb, eb, name=name)
    # The arrays view C memory: free it when the Graph object goes away.
    weakref.finalize(g, lib.gg_free, holder)
    return g


def _check(rc: int, what: str):
    if rc == -2:
        raise MemoryError("graphgen: out of host memory in " + what)
    if rc != 0:
        raise ValueError("graphgen: invalid arguments to %s (rc=%d)" % (what, rc))


def planted(n: int, k: int, p_in: float, inter_pairs: int, seed: int, wmin: int = 1,
            wmax: int = 0) -> Graph:
    """Planted partition: k consecutive blocks, intra pairs with prob p_in,
    `inter_pairs` uniform inter-block pairs.  wmax == 0 -> unit weights (None)."""
    st = _GG()
    _check(_load().gg_planted(n, k, p_in, inter_pairs, wmin, wmax, seed, ctypes.byref(st)), "planted")
    return _wrap(st, "planted(n=%d,k=%d)" % (n, k))


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19, permute=True,
         wmin: int = 1, wmax: int = 0) -> Graph:
    """R-MAT, symmetrised, deduplicated, self loops removed."""
    st = _GG()
    _check(_load().gg_rmat(scale, edge_factor, a, b, c, int(bool(permute)), wmin, wmax, seed,
                           ctypes.byref(st)), "rmat")
    return _wrap(st, "rmat(s=%d,ef=%d)" % (scale, edge_factor))


def road_knn(n: int, k: int, seed: int) -> Graph:
    """2-D random geometric graph, union-symmetrised k nearest neighbours."""
    st = _GG()
    _check(_load().gg_road_knn(n, k, seed, ctypes.byref(st)), "road_knn")
    return _wrap(st, "road_knn(n=%d,k=%d)" % (n, k))


def batched_planted(num_graphs: int, seed: int, nmin=200, nmax=200_000, kmin=5, kmax=500,
                    dmin=8.0, dmax=32.0, inter_deg=2.0) -> Graph:
    """Concatenated batch of planted graphs (local ids per graph)."""
    st = _GG()
    _check(_load().gg_batched_planted(num_graphs, nmin, nmax, kmin, kmax, dmin, dmax, inter_deg,
                                      seed, ctypes.byref(st)), "batched_planted")
    return _wrap(st, "batched_planted(%d)" % num_graphs)


# ----------------------------------------------------------------------------
# Small hand-made graphs (numpy).  Unlike the generators above these keep
# whatever the caller gives them: duplicates, self loops, zero weights.
# ----------------------------------------------------------------------------

def from_entries(n: int, rows, cols, weights=None, name="entries") -> Graph:
    """CSR from directed entries exactly as given (stable by row, then input order)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.argsort(rows, kind="stable")
    counts = np.bincount(rows, minlength=n) if rows.size else np.zeros(n, dtype=np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    w = None
    if weights is not None:
        w = np.asarray(weights, dtype=np.uint32)[order].copy()
    return Graph(off, cols[order].astype(np.int32), w, name=name)


def from_undirected(n: int, edges, weights=None, name="undirected") -> Graph:
    """Symmetric CSR from undirected edges [(u, v), ...]; each edge is stored
    in both rows (a self loop (u, u) once).  Duplicates are kept."""
    rows, cols, ws = [], [], []
    for t, (u, v) in enumerate(edges):
        w = 1 if weights is None else int(weights[t])
        rows.append(u); cols.append(v); ws.append(w)
        if u != v:
            rows.append(v); cols.append(u); ws.append(w)
    return from_entries(n, rows, cols, None if weights is None else ws, name=name)


def from_adjacency(A: np.ndarray, name="adjacency") -> Graph:
    """Symmetric CSR from a dense symmetric weight matrix (0 = no edge)."""
    A = np.asarray(A)
    n = A.shape[0]
    r, c = np.nonzero(A)
    return from_entries(n, r, c, A[r, c].astype(np.uint32), name=name)


def cliques(sizes, perm=None, name="cliques") -> Graph:
    """Disjoint cliques of the given sizes; optional vertex relabelling perm
    (new_id = perm[old_id])."""
    edges = []
    base = 0
    for s in sizes:
        for a in range(s):
            for b in range(a + 1, s):
                edges.append((base + a, base + b))
        base += s
    if perm is not None:
        edges = [(int(perm[u]), int(perm[v])) for u, v in edges]
    return from_undirected(base, edges, name=name)

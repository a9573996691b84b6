"""Python binding of libgsl_lpa.so: GSL-LPA community detection on MI355X.

The functions keep the names of the C ABI (include/gsl_lpa.h) and only marshal
arguments: every step runs in the library's HIP kernels.  Tensors are torch
device tensors (int64 offsets, int32 cols, uint32-valued weights stored as
torch.int32 or torch.uint32, int32 labels) and calls run on torch's current
stream.  If the native library is missing the import fails loudly: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = ["gsl_lpa", "gsl_lpa_ex", "gsl_lpa_f32", "gsl_lpa_batched", "gsl_lpa_graphs", "gsl_check_graph", "Context",
           "gsl_split", "gsl_split_ex", "gsl_disconnected", "gsl_set_tiers", "gsl_get_tiers",
           "gsl_tier_variants",
           "gsl_modularity", "gsl_convergence_limit", "gsl_set_stream", "gsl_release", "gsl_version",
           "GslError", "LIB_PATH", "load"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgsl_lpa.so")
STATS_MAX_ITERS = 64
STATS_TIERS = 10

GSL_OK, GSL_EINVAL, GSL_ENOMEM, GSL_EDEVICE, GSL_EOVERFLOW = 0, -1, -2, -3, -4


class GslError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gsl error %d: %s" % (code, msg))
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("prune", ctypes.c_int32), ("split", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("layout", ctypes.c_int32), ("async_sweeps", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("split_rounds", ctypes.c_int32),
                ("changed", ctypes.c_int64 * STATS_MAX_ITERS),
                ("processed", ctypes.c_int64 * STATS_MAX_ITERS),
                ("edges", ctypes.c_int64 * STATS_MAX_ITERS),
                ("marked", ctypes.c_int64 * STATS_MAX_ITERS),
                ("nnz", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("ms_plan", ctypes.c_float), ("ms_sweeps", ctypes.c_float),
                ("ms_split", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("ms_sweep", ctypes.c_float * STATS_MAX_ITERS),
                ("tier_vertices", ctypes.c_int64 * STATS_TIERS),
                ("tier_launches", ctypes.c_int64 * STATS_TIERS),
                ("tier_processed", ctypes.c_int64 * STATS_TIERS),
                ("tier_edges", ctypes.c_int64 * STATS_TIERS),
                ("tier_changed", ctypes.c_int64 * STATS_TIERS),
                ("tier_marked", ctypes.c_int64 * STATS_TIERS),
                ("tier_sparse", ctypes.c_int64 * STATS_TIERS),
                ("renumbered", ctypes.c_int32), ("ms_reorder", ctypes.c_float),
                ("ms_hub_finish", ctypes.c_float),
                ("ms_tier", ctypes.c_float * STATS_TIERS),
                ("tier_frontier", ctypes.c_int64 * STATS_TIERS),
                ("tier_frontier_listed", ctypes.c_int64 * STATS_TIERS)]


TIER_LEVELS = 7


class _Tier(ctypes.Structure):
    _fields_ = [("max_degree", ctypes.c_int32), ("variant", ctypes.c_int32)]


class _VariantInfo(ctypes.Structure):
    _fields_ = [("group", ctypes.c_int32), ("table_log2", ctypes.c_int32), ("block", ctypes.c_int32),
                ("per_lane", ctypes.c_int32), ("capacity", ctypes.c_int32)]


class _Graph(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("cols", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("labels_out", ctypes.c_void_p), ("n", ctypes.c_int64)]


_lib = None
_VP = ctypes.c_void_p


def load(path: str = None):
    """Loads the native library (raises if it was not built).  The path
    defaults to the in-tree build; GSL_LPA_LIB may name another build."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("GSL_LPA_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError("libgsl_lpa.so not found at %s: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % path)
    lib = ctypes.CDLL(path)
    lib.gsl_lpa.argtypes = [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, _VP]
    lib.gsl_lpa_ex.argtypes = [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                               ctypes.POINTER(_Options), ctypes.POINTER(_Stats), _VP]
    lib.gsl_lpa_batched.argtypes = [ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32,
                                    ctypes.c_double, _VP]
    lib.gsl_lpa_batched_ex.argtypes = [ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, ctypes.c_int32,
                                       ctypes.c_double, ctypes.POINTER(_Options), ctypes.POINTER(_Stats),
                                       _VP, _VP]
    lib.gsl_context_create.argtypes = [ctypes.POINTER(_VP)]
    lib.gsl_context_destroy.argtypes = [_VP]
    lib.gsl_context_destroy.restype = None
    lib.gsl_context_set_stream.argtypes = [_VP, _VP]
    lib.gsl_context_stream.argtypes = [_VP]
    lib.gsl_context_stream.restype = _VP
    lib.gsl_lpa_graphs.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(_Graph), ctypes.c_int32,
                                   ctypes.c_double, ctypes.POINTER(_Options), ctypes.POINTER(_Stats),
                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.gsl_check_graph.argtypes = [_VP, _VP, ctypes.c_int64]
    lib.gsl_lpa_f32.argtypes = [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
                                ctypes.POINTER(_Options), ctypes.POINTER(_Stats), _VP]
    lib.gsl_set_tiers.argtypes = [ctypes.POINTER(_Tier)]
    lib.gsl_get_tiers.argtypes = [ctypes.POINTER(_Tier)]
    lib.gsl_tier_variant.argtypes = [ctypes.c_int32, ctypes.POINTER(_VariantInfo)]
    lib.gsl_disconnected.argtypes = [_VP, _VP, ctypes.c_int64, _VP, _VP, ctypes.POINTER(ctypes.c_int64)]
    lib.gsl_split_ex.argtypes = [_VP, _VP, ctypes.c_int64, _VP, _VP, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float)]
    lib.gsl_split.argtypes = [_VP, _VP, ctypes.c_int64, _VP, _VP]
    lib.gsl_modularity.argtypes = [_VP, _VP, _VP, ctypes.c_int64, _VP, ctypes.POINTER(ctypes.c_double)]
    lib.gsl_convergence_limit.argtypes = [ctypes.c_int64, ctypes.c_double]
    lib.gsl_convergence_limit.restype = ctypes.c_int64
    lib.gsl_set_hub_limits.argtypes = [ctypes.c_int64, ctypes.c_int32]
    lib.gsl_lpa_noalloc.argtypes = [_VP, _VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, _VP]
    lib.gsl_graphs_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    lib.gsl_graphs_bytes.restype = ctypes.c_int64
    lib.gsl_session_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
    lib.gsl_session_bytes.restype = ctypes.c_int64
    lib.gsl_session_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_int32, ctypes.POINTER(_VP)]
    lib.gsl_session_destroy.argtypes = [_VP]
    lib.gsl_session_destroy.restype = None
    lib.gsl_session_stream.argtypes = [_VP]
    lib.gsl_session_stream.restype = _VP
    lib.gsl_session_add.argtypes = [_VP, ctypes.c_int64, ctypes.POINTER(_Graph), ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.gsl_session_step.argtypes = [_VP, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    lib.gsl_session_info.argtypes = [_VP] + [ctypes.POINTER(ctypes.c_int64)] * 6
    lib.gsl_set_stream.argtypes = [_VP]
    lib.gsl_last_error.restype = ctypes.c_char_p
    lib.gsl_version.restype = ctypes.c_char_p
    lib.gsl_release.restype = None
    for f in (lib.gsl_lpa, lib.gsl_lpa_ex, lib.gsl_split, lib.gsl_modularity, lib.gsl_set_stream,
              lib.gsl_lpa_batched, lib.gsl_lpa_batched_ex, lib.gsl_context_create, lib.gsl_context_set_stream,
              lib.gsl_lpa_graphs, lib.gsl_check_graph, lib.gsl_disconnected, lib.gsl_set_tiers,
              lib.gsl_get_tiers, lib.gsl_tier_variant, lib.gsl_split_ex, lib.gsl_lpa_f32,
              lib.gsl_set_hub_limits, lib.gsl_lpa_noalloc, lib.gsl_session_create, lib.gsl_session_add,
              lib.gsl_session_step, lib.gsl_session_info):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != GSL_OK:
        raise GslError(rc, _lib.gsl_last_error().decode())


def _dev(t, dtypes, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise TypeError("%s must be a tensor" % name)
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))
    if not t.is_contiguous():
        raise TypeError("%s must be contiguous" % name)
    return t.data_ptr() if t.numel() else None


_U32 = tuple(d for d in (getattr(torch, "uint32", None), torch.int32) if d is not None)


def _bind_stream():
    lib = load()
    _check(lib.gsl_set_stream(_VP(torch.cuda.current_stream().cuda_stream)))
    return lib


def _graph_args(offsets, cols, weights):
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets must hold n + 1 entries")
    return (_dev(offsets, (torch.int64,), "offsets"), _dev(cols, (torch.int32,), "cols"),
            _dev(weights, _U32, "weights", allow_none=True), n)


def gsl_lpa(offsets, cols, weights=None, max_iters=20, tolerance=0.05, out=None):
    """GSL-LPA labels (int32 tensor).  See include/gsl_lpa.h."""
    labels, _ = gsl_lpa_ex(offsets, cols, weights, max_iters, tolerance, out=out)
    return labels


def gsl_lpa_noalloc(offsets, cols, weights=None, max_iters=20, tolerance=0.05, out=None):
    """gsl_lpa without any device allocation by the library (its scratch is a
    static device array; see include/gsl_lpa.h for the size limits).  `out`
    should be preallocated by callers that must not allocate."""
    lib = _bind_stream()
    po, pc, pw, n = _graph_args(offsets, cols, weights)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=offsets.device)
    if out.numel() != n:
        raise ValueError("out must hold n labels")
    _check(lib.gsl_lpa_noalloc(po, pc, pw, n, int(max_iters), float(tolerance), _dev(out, (torch.int32,), "out")))
    return out


LAYOUTS = {"auto": 0, "renumbered": 1, "original": 2}


def gsl_lpa_ex(offsets, cols, weights=None, max_iters=20, tolerance=0.05, prune=True, split=True,
               timing=False, layout="auto", out=None, async_sweeps=False):
    """Returns (labels, stats dict).  layout: "auto", "renumbered" or
    "original" (which vertex order the sweeps run in; results are identical).
    async_sweeps: the paper's in-place sweeps (results depend on timing)."""
    lib = _bind_stream()
    po, pc, pw, n = _graph_args(offsets, cols, weights)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=offsets.device)
    if out.numel() != n:
        raise ValueError("out must hold n labels")
    pl = _dev(out, (torch.int32,), "out")
    opt = _Options(int(bool(prune)), int(bool(split)), int(bool(timing)), LAYOUTS[layout], int(bool(async_sweeps)))
    st = _Stats()
    _check(lib.gsl_lpa_ex(po, pc, pw, n, int(max_iters), float(tolerance), ctypes.byref(opt),
                          ctypes.byref(st), pl))
    return out, _stats_dict(st)


def _stats_dict(st):
    it = st.iterations
    k = min(it, STATS_MAX_ITERS)
    return {"iterations": it, "changed": list(st.changed[:k]), "processed": list(st.processed[:k]),
            "edges": list(st.edges[:k]), "marked": list(st.marked[:k]), "nnz": st.nnz,
            "max_degree": st.max_degree, "ms_plan": st.ms_plan, "ms_sweeps": st.ms_sweeps,
            "ms_split": st.ms_split, "ms_total": st.ms_total, "ms_sweep": list(st.ms_sweep[:k]),
            "renumbered": bool(st.renumbered), "ms_reorder": st.ms_reorder,
            "ms_hub_finish": st.ms_hub_finish,
            "tiers": [{"vertices": st.tier_vertices[t], "launches": st.tier_launches[t],
                       "processed": st.tier_processed[t], "edges": st.tier_edges[t],
                       "changed": st.tier_changed[t], "marked": st.tier_marked[t],
                       "sparse_launches": st.tier_sparse[t], "frontier_launches": st.tier_frontier[t],
                       "frontier_listed": st.tier_frontier_listed[t], "ms": st.ms_tier[t]}
                      for t in range(STATS_TIERS)]}


def gsl_lpa_f32(offsets, cols, weights=None, max_iters=20, tolerance=0.05, prune=True, split=True, timing=False,
                layout="auto", out=None, async_sweeps=False):
    """gsl_lpa_ex with float32 weights summed in fp64.  Returns (labels, stats)."""
    lib = _bind_stream()
    po, pc, _, n = _graph_args(offsets, cols, None)
    pw = _dev(weights, (torch.float32,), "weights", allow_none=True)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=offsets.device)
    if out.numel() != n:
        raise ValueError("out must hold n labels")
    opt = _Options(int(bool(prune)), int(bool(split)), int(bool(timing)), LAYOUTS[layout], int(bool(async_sweeps)))
    st = _Stats()
    _check(lib.gsl_lpa_f32(po, pc, pw, n, int(max_iters), float(tolerance), ctypes.byref(opt), ctypes.byref(st),
                           _dev(out, (torch.int32,), "out")))
    return out, _stats_dict(st)


def gsl_lpa_batched(vtx_base, edge_base, offsets, cols, weights=None, max_iters=20, tolerance=0.05,
                    prune=True, split=True, timing=False, out=None):
    """A batch of independent graphs as one concatenated CSR (local ids; see
    include/gsl_lpa.h).  Returns (labels, per-graph sweep counts, stats)."""
    lib = _bind_stream()
    G = vtx_base.numel() - 1
    if G < 0 or edge_base.numel() != G + 1:
        raise ValueError("vtx_base and edge_base must hold num_graphs + 1 entries")
    po, pc, pw, n = _graph_args(offsets, cols, weights)
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=offsets.device)
    if out.numel() != n:
        raise ValueError("out must hold N labels")
    iters = torch.zeros(max(G, 0), dtype=torch.int32, device=offsets.device)
    opt = _Options(int(bool(prune)), int(bool(split)), int(bool(timing)), 2, 0)
    st = _Stats()
    _check(lib.gsl_lpa_batched_ex(G, _dev(vtx_base, (torch.int64,), "vtx_base"),
                                  _dev(edge_base, (torch.int64,), "edge_base"), po, pc, pw,
                                  int(max_iters), float(tolerance), ctypes.byref(opt), ctypes.byref(st),
                                  _dev(out, (torch.int32,), "out"),
                                  _dev(iters, (torch.int32,), "iters") if G else None))
    return out, iters, _stats_dict(st)


def _graph_table(graphs):
    tab = (_Graph * max(len(graphs), 1))()
    outs = []
    for k, gr in enumerate(graphs):
        offsets, cols, weights = gr[0], gr[1], gr[2] if len(gr) > 2 else None
        out = gr[3] if len(gr) > 3 and gr[3] is not None else None
        n = offsets.numel() - 1
        if n < 0:
            raise ValueError("graph %d: offsets must hold n + 1 entries" % k)
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=offsets.device)
        if out.numel() != n:
            raise ValueError("graph %d: out must hold n labels" % k)
        tab[k].offsets = _dev(offsets, (torch.int64,), "offsets")
        tab[k].cols = _dev(cols, (torch.int32,), "cols")
        tab[k].weights = _dev(weights, _U32, "weights", allow_none=True)
        tab[k].labels_out = _dev(out, (torch.int32,), "out")
        tab[k].n = n
        outs.append(out)
    return tab, outs


def gsl_lpa_graphs(graphs, max_iters=20, tolerance=0.05, prune=True, split=True, ctx=None,
                   return_status=False):
    """A batch of separate graphs: graphs is a list of (offsets, cols[,
    weights[, out]]) tensors.  Returns (list of labels, list of sweep counts,
    stats), plus the list of per-graph statuses if return_status (a malformed
    graph then gets GSL_EINVAL there instead of failing the call).  ctx: a
    Context (its own scratch and stream) or None."""
    if ctx is not None:
        return ctx.lpa_graphs(graphs, max_iters, tolerance, prune, split, return_status)
    lib = _bind_stream()
    return _run_graphs(lib, None, graphs, max_iters, tolerance, prune, split, return_status)


def _run_graphs(lib, handle, graphs, max_iters, tolerance, prune, split, return_status=False):
    tab, outs = _graph_table(graphs)
    G = len(graphs)
    iters = (ctypes.c_int32 * max(G, 1))()
    status = (ctypes.c_int32 * max(G, 1))() if return_status else None
    opt = _Options(int(bool(prune)), int(bool(split)), 0, 2, 0)
    st = _Stats()
    _check(lib.gsl_lpa_graphs(handle, G, tab, int(max_iters), float(tolerance), ctypes.byref(opt),
                              ctypes.byref(st), iters, status))
    if return_status:
        return outs, list(iters[:G]), _stats_dict(st), list(status[:G])
    return outs, list(iters[:G]), _stats_dict(st)


def gsl_check_graph(offsets, cols) -> None:
    """Raises GslError(GSL_EINVAL) unless offsets start at 0, never decrease
    and every column is in [0, n)."""
    lib = _bind_stream()
    po, pc, _, n = _graph_args(offsets, cols, None)
    _check(lib.gsl_check_graph(po, pc, n))


class Context:
    """Scratch memory and a stream of its own (gsl_context).  Calls on
    different contexts may run at once from different threads; ctypes drops
    the GIL during the call, so their work overlaps on the device."""

    def __init__(self):
        self._lib = load()
        h = _VP()
        _check(self._lib.gsl_context_create(ctypes.byref(h)))
        self._h = h
        self.stream = torch.cuda.ExternalStream(self._lib.gsl_context_stream(h))

    def lpa_graphs(self, graphs, max_iters=20, tolerance=0.05, prune=True, split=True, return_status=False):
        if self._h is None:
            raise RuntimeError("context closed")
        # inputs written on torch's current stream must be ready first
        self.stream.wait_stream(torch.cuda.current_stream())
        return _run_graphs(self._lib, self._h, graphs, max_iters, tolerance, prune, split, return_status)

    def close(self):
        if self._h is not None:
            self._lib.gsl_context_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


GSL_EAGAIN = -5


def gsl_graphs_bytes(n, nnz, graphs=1, weighted=False, max_iters=20) -> int:
    """Upper bound of the device scratch a gsl_lpa_graphs call on a batch of
    that size adds (library query, host only)."""
    return int(load().gsl_graphs_bytes(int(n), int(nnz), int(graphs), int(bool(weighted)), int(max_iters)))


class Session:
    """Continuous batching (gsl_session): a resident batch that graphs join
    and leave between sweeps.  add() admits graphs (lists of (offsets, cols[,
    weights[, out]]) tensors) and returns (ticket, status, out) per graph;
    step(sweeps) runs that many sweeps of every resident graph and returns
    [(ticket, sweeps_run)] of the graphs that finished, whose labels are then
    in their out tensors.  Each result equals gsl_lpa on the graph alone."""

    def __init__(self, max_vertices, max_entries, max_graphs=1024, max_iters=20, tolerance=0.05,
                 weighted=False):
        self._lib = load()
        h = _VP()
        _check(self._lib.gsl_session_create(int(max_vertices), int(max_entries), int(max_graphs), int(max_iters),
                                            float(tolerance), int(bool(weighted)), ctypes.byref(h)))
        self._h = h
        self.max_graphs = int(max_graphs)
        self.stream = torch.cuda.ExternalStream(self._lib.gsl_session_stream(h))
        # output tensors of the running graphs, held until their graph
        # finishes (the session writes them at the end of a later step)
        self._outs = {}

    @staticmethod
    def device_bytes(max_vertices, max_entries, max_graphs=1024, weighted=False) -> int:
        """Device bytes a session of this capacity holds (library query)."""
        return int(load().gsl_session_bytes(int(max_vertices), int(max_entries), int(max_graphs),
                                            int(bool(weighted))))

    def add(self, graphs):
        if self._h is None:
            raise RuntimeError("session closed")
        G = len(graphs)
        if G == 0:
            return []
        tab, outs = _graph_table(graphs)
        tickets = (ctypes.c_int64 * G)()
        status = (ctypes.c_int32 * G)()
        self.stream.wait_stream(torch.cuda.current_stream())
        _check(self._lib.gsl_session_add(self._h, G, tab, tickets, status))
        for k in range(G):
            if tickets[k] >= 0:
                self._outs[tickets[k]] = outs[k]
        return [(tickets[k], status[k], outs[k]) for k in range(G)]

    def step(self, sweeps=1, capacity=None):
        if self._h is None:
            raise RuntimeError("session closed")
        cap = int(capacity if capacity is not None else self.max_graphs)
        t = (ctypes.c_int64 * max(cap, 1))()
        it = (ctypes.c_int32 * max(cap, 1))()
        cnt = ctypes.c_int64(0)
        _check(self._lib.gsl_session_step(self._h, int(sweeps), cap, t, it, ctypes.byref(cnt)))
        for k in range(cnt.value):
            self._outs.pop(t[k], None)
        return [(t[k], it[k]) for k in range(cnt.value)]

    def info(self):
        vals = [ctypes.c_int64(0) for _ in range(6)]
        _check(self._lib.gsl_session_info(self._h, *[ctypes.byref(v) for v in vals]))
        keys = ("live_graphs", "live_vertices", "live_entries", "free_vertices", "free_entries", "device_bytes")
        return {k: v.value for k, v in zip(keys, vals)}

    def close(self):
        if self._h is not None:
            self._lib.gsl_session_destroy(self._h)
            self._h = None
            self._outs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gsl_split(offsets, cols, labels_in, out=None):
    lib = _bind_stream()
    po, pc, _, n = _graph_args(offsets, cols, None)
    if labels_in.numel() != n:
        raise ValueError("labels_in must hold n labels")
    pin = _dev(labels_in, (torch.int32,), "labels_in")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=offsets.device)
    _check(lib.gsl_split(po, pc, n, pin, _dev(out, (torch.int32,), "out")))
    return out


SPLIT_TECHNIQUES = {"union-find": 0, "lp": 1, "lpp": 2}


def gsl_split_ex(offsets, cols, labels_in, technique="union-find", out=None):
    """The split with a chosen technique ("union-find", "lp", "lpp"; same
    labels).  Returns (labels, rounds, device ms)."""
    lib = _bind_stream()
    po, pc, _, n = _graph_args(offsets, cols, None)
    if labels_in.numel() != n:
        raise ValueError("labels_in must hold n labels")
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=offsets.device)
    rounds, ms = ctypes.c_int32(0), ctypes.c_float(0.0)
    _check(lib.gsl_split_ex(po, pc, n, _dev(labels_in, (torch.int32,), "labels_in"),
                            _dev(out, (torch.int32,), "out"), SPLIT_TECHNIQUES[technique], ctypes.byref(rounds),
                            ctypes.byref(ms)))
    return out, rounds.value, ms.value


def gsl_disconnected(offsets, cols, labels, flags=True):
    """Alg. 4: (number of disconnected communities, uint8 flags indexed by
    label or None)."""
    lib = _bind_stream()
    po, pc, _, n = _graph_args(offsets, cols, None)
    if labels.numel() != n:
        raise ValueError("labels must hold n labels")
    D = torch.empty(n, dtype=torch.uint8, device=offsets.device) if flags else None
    cnt = ctypes.c_int64(0)
    _check(lib.gsl_disconnected(po, pc, n, _dev(labels, (torch.int32,), "labels"),
                                _dev(D, (torch.uint8,), "flags", allow_none=True), ctypes.byref(cnt)))
    return cnt.value, D


def gsl_modularity(offsets, cols, weights, labels) -> float:
    lib = _bind_stream()
    po, pc, pw, n = _graph_args(offsets, cols, weights)
    if labels.numel() != n:
        raise ValueError("labels must hold n labels")
    q = ctypes.c_double(0.0)
    _check(lib.gsl_modularity(po, pc, pw, n, _dev(labels, (torch.int32,), "labels"), ctypes.byref(q)))
    return q.value


def gsl_set_tiers(levels=None) -> None:
    """Degree tiers of later calls: a list of TIER_LEVELS (max_degree,
    variant) pairs, or None for the defaults.  Changes speed, not results."""
    lib = load()
    if levels is None:
        _check(lib.gsl_set_tiers(None))
        return
    if len(levels) != TIER_LEVELS:
        raise ValueError("need %d levels" % TIER_LEVELS)
    arr = (_Tier * TIER_LEVELS)(*[_Tier(int(d), int(v)) for d, v in levels])
    _check(lib.gsl_set_tiers(arr))


def gsl_get_tiers():
    lib = load()
    arr = (_Tier * TIER_LEVELS)()
    _check(lib.gsl_get_tiers(arr))
    return [(t.max_degree, t.variant) for t in arr]


def gsl_tier_variants():
    """Shapes of the sweep kernel variants: list of dicts (index = variant)."""
    lib = load()
    out = []
    while True:
        info = _VariantInfo()
        if lib.gsl_tier_variant(len(out), ctypes.byref(info)) != GSL_OK:
            return out
        out.append({"group": info.group, "table_log2": info.table_log2, "block": info.block,
                    "per_lane": info.per_lane, "capacity": info.capacity})


def variant_kernel_name(v: dict, weighted: bool = False, n: int = 0, aligned: bool = True) -> str:
    """The sweep kernel's name as profilers print it (template arguments;
    the thread variants have weighted and unit-weight kernels, each with
    32-bit gather offsets for fewer than 2^30 vertices or 64-bit ones, and
    16-byte row loads when the column and weight arrays are 16-byte aligned,
    as the library's own copies always are)."""
    if v["group"] == 1:
        t = lambda x: "true" if x else "false"  # noqa: E731
        return "sweep_thread<%d, %s, %s, %s>" % (v["per_lane"], t(weighted), t(n < (1 << 30)), t(aligned))
    return "sweep_lds<%d, %d, %d, %d>" % (v["group"], v["table_log2"], v["block"], v["per_lane"])


def gsl_set_hub_limits(staging_bytes: int = 0, merge_claims: int = 0) -> None:
    """Hub tier limits of later calls: staging bytes per hub batch and the
    distinct labels one merge pass accepts (0: the defaults).  Changes memory
    use and speed, not results."""
    _check(load().gsl_set_hub_limits(int(staging_bytes), int(merge_claims)))


def gsl_convergence_limit(n: int, tolerance: float) -> int:
    return int(load().gsl_convergence_limit(int(n), float(tolerance)))


def gsl_set_stream(stream) -> None:
    _check(load().gsl_set_stream(_VP(stream.cuda_stream if hasattr(stream, "cuda_stream") else stream)))


def gsl_release() -> None:
    load().gsl_release()


def gsl_version() -> str:
    return load().gsl_version().decode()

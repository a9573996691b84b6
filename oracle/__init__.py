"""GSL-LPA oracle: plain single-threaded CPU reference (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it, and it shares no code
with the GPU path.  The arithmetic lives in ``gsl_oracle.cpp`` (built with g++
into ``liboracle.so``); this module only marshals numpy arrays.

Functions follow arXiv:2403.01261:
  lpa           Alg. 3 (synchronous sweeps, pruning, Eq. 2 label rule) + Alg. 2
  lpa_f32       the same with fp32 weights summed in fp64
  split_bfs     Alg. 2
  split_lp      Alg. 1 (LP / LPP)
  modularity    Eq. 1 (second form)
  disconnected  Alg. 4
Every function is pinned by the ``-m "not gpu"`` tests (brute force on tiny
graphs, closed forms, invariants); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsl_oracle.cpp")
_LIB = os.environ.get("GSL_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wno-stringop-overflow",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_P64 = ctypes.POINTER(ctypes.c_int64)
_P32 = ctypes.POINTER(ctypes.c_int32)
_PU32 = ctypes.POINTER(ctypes.c_uint32)
_PU64 = ctypes.POINTER(ctypes.c_uint64)
_PU8 = ctypes.POINTER(ctypes.c_uint8)
_PF32 = ctypes.POINTER(ctypes.c_float)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_lpa.argtypes = [ctypes.c_int64, _P64, _P32, _PU32, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int, _P32, _P32, _P64, _P32, _P64]
        lib.oracle_split_bfs.argtypes = [ctypes.c_int64, _P64, _P32, _P32, _P32]
        lib.oracle_split_lp.argtypes = [ctypes.c_int64, _P64, _P32, _P32, ctypes.c_int, _P32, _P64]
        lib.oracle_modularity.argtypes = [ctypes.c_int64, _P64, _P32, _PU32, _P32,
                                          ctypes.POINTER(ctypes.c_double), _PU64]
        lib.oracle_disconnected.argtypes = [ctypes.c_int64, _P64, _P32, _P32, _PU8, _P64]
        lib.oracle_lpa_f32.argtypes = [ctypes.c_int64, _P64, _P32, _PF32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_int, ctypes.c_int, _P32, ctypes.POINTER(ctypes.c_int32), _P64,
                                       _P32, _P64]
        lib.oracle_lpa_f32.restype = ctypes.c_int
        for f in (lib.oracle_lpa, lib.oracle_split_bfs, lib.oracle_split_lp, lib.oracle_modularity,
                  lib.oracle_disconnected):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a, typ):
    if a is None:
        return None
    return a.ctypes.data_as(typ)


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    cols = np.ascontiguousarray(g.cols, dtype=np.int32)
    w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.uint32)
    return off, cols, w


def _rc(rc, what):
    if rc == -1:
        raise ValueError("oracle.%s: invalid arguments" % what)
    if rc != 0:
        raise MemoryError("oracle.%s: failed (rc=%d)" % (what, rc))


class LpaResult:
    def __init__(self, labels, iterations, dn, history, processed):
        self.labels = labels          # int32[n]
        self.iterations = iterations  # sweeps performed
        self.dn = dn                  # int64[iterations]: changed vertices per sweep
        self.history = history        # int32[iterations, n] or None
        self.processed = processed    # int64[iterations]: vertices scanned per sweep


def lpa(g, max_iters=20, tolerance=0.05, prune=True, split=True, history=False) -> LpaResult:
    off, cols, w = _csr(g)
    n = off.shape[0] - 1
    labels = np.empty(n, dtype=np.int32)
    iters = ctypes.c_int32(0)
    dn = np.zeros(max(max_iters, 1), dtype=np.int64)
    proc = np.zeros(max(max_iters, 1), dtype=np.int64)
    hist = np.empty((max_iters, n), dtype=np.int32) if history else None
    _rc(_load().oracle_lpa(n, _ptr(off, _P64), _ptr(cols, _P32), _ptr(w, _PU32), max_iters,
                           float(tolerance), int(bool(prune)), int(bool(split)),
                           _ptr(labels, _P32), ctypes.byref(iters), _ptr(dn, _P64),
                           _ptr(hist, _P32), _ptr(proc, _P64)), "lpa")
    it = iters.value
    return LpaResult(labels, it, dn[:it].copy(), None if hist is None else hist[:it].copy(),
                     proc[:it].copy())


def lpa_f32(g, weights, max_iters=20, tolerance=0.05, prune=True, split=True) -> LpaResult:
    """lpa with fp32 weights (float32 array, one per CSR entry; None = unit)
    summed in fp64 in CSR entry order."""
    off, cols, _ = _csr(g)
    n = off.shape[0] - 1
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    labels = np.empty(n, dtype=np.int32)
    iters = ctypes.c_int32(0)
    dn = np.zeros(max(max_iters, 1), dtype=np.int64)
    proc = np.zeros(max(max_iters, 1), dtype=np.int64)
    _rc(_load().oracle_lpa_f32(n, _ptr(off, _P64), _ptr(cols, _P32), _ptr(w, _PF32), max_iters, float(tolerance),
                               int(bool(prune)), int(bool(split)), _ptr(labels, _P32), ctypes.byref(iters),
                               _ptr(dn, _P64), None, _ptr(proc, _P64)), "lpa_f32")
    it = iters.value
    return LpaResult(labels, it, dn[:it].copy(), None, proc[:it].copy())


def split_bfs(g, labels) -> np.ndarray:
    off, cols, _ = _csr(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty(off.shape[0] - 1, dtype=np.int32)
    _rc(_load().oracle_split_bfs(off.shape[0] - 1, _ptr(off, _P64), _ptr(cols, _P32),
                                 _ptr(lab, _P32), _ptr(out, _P32)), "split_bfs")
    return out


def split_lp(g, labels, prune=True):
    off, cols, _ = _csr(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty(off.shape[0] - 1, dtype=np.int32)
    rounds = ctypes.c_int64(0)
    _rc(_load().oracle_split_lp(off.shape[0] - 1, _ptr(off, _P64), _ptr(cols, _P32),
                                _ptr(lab, _P32), int(bool(prune)), _ptr(out, _P32),
                                ctypes.byref(rounds)), "split_lp")
    return out, rounds.value


def modularity(g, labels, parts=False):
    off, cols, w = _csr(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    q = ctypes.c_double(0.0)
    p = np.zeros(4, dtype=np.uint64)
    _rc(_load().oracle_modularity(off.shape[0] - 1, _ptr(off, _P64), _ptr(cols, _P32),
                                  _ptr(w, _PU32), _ptr(lab, _P32), ctypes.byref(q),
                                  _ptr(p, _PU64)), "modularity")
    if parts:
        two_m, I = int(p[0]), int(p[1])
        S2 = int(p[2]) + (int(p[3]) << 64)
        return q.value, (two_m, I, S2)
    return q.value


def disconnected(g, labels):
    """Alg. 4: returns (D uint8[n] indexed by label, count)."""
    off, cols, _ = _csr(g)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    n = off.shape[0] - 1
    D = np.zeros(n, dtype=np.uint8)
    cnt = ctypes.c_int64(0)
    _rc(_load().oracle_disconnected(n, _ptr(off, _P64), _ptr(cols, _P32), _ptr(lab, _P32),
                                    _ptr(D, _PU8), ctypes.byref(cnt)), "disconnected")
    return D, cnt.value

"""Dense brute-force references for tiny graphs (independent of the oracle).

Everything here works on dense matrices batched over many graphs at once:
  W[b, i, j]  summed weight of the entries (i, j) of graph b
  X[b, i, j]  True iff graph b has at least one entry (i, j)
Label weights come from a matrix product with a one-hot label matrix, the
argmax from numpy (first maximum = smallest label), connectivity from
repeated boolean squaring of the intra-community adjacency.  None of it
shares an algorithm with the oracle's sparse accumulator, BFS or union-find.
"""
from __future__ import annotations

import itertools

import numpy as np


def all_graphs(n: int) -> np.ndarray:
    """Adjacency (bool[B, n, n]) of every simple undirected graph on n vertices."""
    pairs = list(itertools.combinations(range(n), 2))
    B = 1 << len(pairs)
    bits = (np.arange(B, dtype=np.int64)[:, None] >> np.arange(len(pairs))) & 1
    A = np.zeros((B, n, n), dtype=bool)
    for t, (u, v) in enumerate(pairs):
        A[:, u, v] = bits[:, t].astype(bool)
        A[:, v, u] = A[:, u, v]
    return A


def label_weights(W: np.ndarray, X: np.ndarray, L: np.ndarray):
    """Per (graph, vertex, label): summed weight and candidate flag, self
    entries excluded."""
    B, n, _ = W.shape
    eye = np.eye(n, dtype=bool)[None]
    dt = np.float64 if np.issubdtype(W.dtype, np.floating) else np.int64  # float weights: fp64 sums
    Wn = np.where(eye, 0, W).astype(dt)
    Xn = X & ~eye
    onehot = (L[:, :, None] == np.arange(n)[None, None, :]).astype(dt)  # [B, j, c]
    S = Wn @ onehot                       # [B, i, c] summed weight per label
    cand = (Xn.astype(np.int64) @ onehot) > 0
    return S, cand


def best_labels(W, X, L):
    """Eq. 2 with smallest-label tie-break; vertices with no candidate keep L."""
    S, cand = label_weights(W, X, L)
    score = np.where(cand, S, -1)
    best = np.argmax(score, axis=2)
    has = cand.any(axis=2)
    return np.where(has, best, L)


def lpa(W, X, max_iters, tol):
    """Synchronous LPA over a batch; each graph stops on its own when
    changed/N <= tol.  Returns (labels[B, n], iterations[B], dn list of
    per-sweep arrays, history list)."""
    B, n, _ = W.shape
    L = np.tile(np.arange(n, dtype=np.int64), (B, 1))
    done = np.zeros(B, dtype=bool)
    iters = np.zeros(B, dtype=np.int64)
    dns, hist = [], []
    for _ in range(max_iters):
        if done.all():
            break
        nl = best_labels(W, X, L)
        nl = np.where(done[:, None], L, nl)
        dn = (nl != L).sum(axis=1)
        dn = np.where(done, -1, dn)
        L = nl
        iters += ~done
        dns.append(dn)
        hist.append(L.copy())
        done = done | ((dn >= 0) & (dn / n <= tol))
    return L, iters, dns, hist


def closure(R: np.ndarray) -> np.ndarray:
    """Reflexive-transitive closure of bool[B, n, n] by repeated squaring."""
    B, n, _ = R.shape
    R = R | np.eye(n, dtype=bool)[None]
    steps = max(1, int(np.ceil(np.log2(max(n, 2)))))
    for _ in range(steps + 1):
        Ri = R.astype(np.int64)
        R = (Ri @ Ri) > 0
    return R


def split(X, L):
    """Smallest vertex id reachable inside the own community (Alg. 2 output)."""
    B, n, _ = X.shape
    same = L[:, :, None] == L[:, None, :]
    R = closure(X & same)
    idx = np.arange(n)[None, None, :]
    return np.where(R, idx, n).min(axis=2)


def components_per_label(X, L):
    """Number of connected pieces of every label (bool adjacency, one graph)."""
    n = X.shape[0]
    reach = closure((X & (L[:, None] == L[None, :]))[None])[0]
    rep = np.where(reach, np.arange(n)[None, :], n).min(axis=1)
    out = {}
    for c in np.unique(L):
        out[int(c)] = len(np.unique(rep[L == c]))
    return out


def modularity_pairs(W, L):
    """Eq. 1 first form, with the null-model term over ALL ordered vertex
    pairs: Q = 1/2m * sum_{i,j} [W_ij - K_i K_j / 2m] delta(C_i, C_j)."""
    W = W.astype(np.float64)
    K = W.sum(axis=1)
    two_m = W.sum()
    if two_m == 0:
        return 0.0
    same = L[:, None] == L[None, :]
    return float(((W - np.outer(K, K) / two_m) * same).sum() / two_m)


def dense_from_graph(g):
    """Dense (W, X) of one CSR graph (duplicates summed)."""
    n = g.n
    W = np.zeros((n, n), dtype=np.int64)
    X = np.zeros((n, n), dtype=bool)
    rows = np.repeat(np.arange(n), np.diff(g.offsets))
    w = np.ones(g.nnz, dtype=np.int64) if g.weights is None else g.weights.astype(np.int64)
    np.add.at(W, (rows, g.cols.astype(np.int64)), w)
    X[rows, g.cols] = True
    return W, X

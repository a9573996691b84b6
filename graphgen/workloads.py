"""The five synthetic workloads (stand-ins for the paper's SuiteSparse graphs).

Seeds are 240301261 + workload number (1..5).  All graphs are symmetric,
deduplicated, self-loop free CSR with int32 columns and int64 offsets.

  1  planted-10k      planted partition, 10,000 vertices in 100 blocks of 100,
                      intra-pair prob 0.1, 10,000 uniform inter-block pairs
                      (mean inter-degree 2), unit weights
  2  rmat-s22         R-MAT scale 22, edge factor 16, a/b/c/d = .57/.19/.19/.05,
                      random vertex relabelling, weights uniform in [1, 16]
  3  road-24m         24M points uniform in the unit square, union-symmetrised
                      2-nearest-neighbour graph (mean degree ~2.58), unit weights
  4  rmat-s26         R-MAT scale 26, edge factor 32, same a/b/c/d and
                      relabelling, unit weights
  5  batched-4096     4,096 planted graphs, N log-uniform in [200, 200,000],
                      5-500 blocks (at most N/10), target mean degree U[8, 32]
                      with inter-degree 2, unit weights, local ids per graph

Every workload also has a reduced form (`small=True`) of the same family, used
where a test must finish in seconds.
"""
from __future__ import annotations

import os

import numpy as np

from . import Graph, batched_planted, planted, rmat, road_knn

SEED_BASE = 240301261

NAMES = {1: "planted-10k", 2: "rmat-s22", 3: "road-24m", 4: "rmat-s26", 5: "batched-4096"}

# Sweep parameters used for every workload: MAX_ITERATIONS and tau.
MAX_ITERS = 20
TOLERANCE = 0.05


def make(idx: int, small: bool = False):
    """Workload idx.  With GSL_GRAPH_CACHE set to a directory, the arrays are
    kept there as .npy files after the first generation and loaded by later
    calls (several processes of one session then generate a large graph once)."""
    cache = os.environ.get("GSL_GRAPH_CACHE")
    if not cache:
        return _generate(idx, small)
    stem = os.path.join(cache, describe(idx, small))
    parts = ("offsets", "cols", "weights", "vtx_base", "edge_base")
    if os.path.exists(stem + ".done"):
        arrs = {k: (np.load(stem + "." + k + ".npy") if os.path.exists(stem + "." + k + ".npy") else None)
                for k in parts}
        return Graph(arrs["offsets"], arrs["cols"], arrs["weights"], arrs["vtx_base"], arrs["edge_base"],
                     name=describe(idx, small))
    g = _generate(idx, small)
    try:
        os.makedirs(cache, exist_ok=True)
        for k in parts:
            a = getattr(g, k)
            if a is not None:
                np.save(stem + "." + k + ".npy", a)
        open(stem + ".done", "w").close()
    except OSError:
        pass  # no room: later calls generate again
    return g


def _generate(idx: int, small: bool):
    seed = SEED_BASE + idx
    if idx == 1:
        return planted(10_000, 100, 0.1, 10_000, seed)
    if idx == 2:
        if small:
            return rmat(14, 16, seed, wmin=1, wmax=16)
        return rmat(22, 16, seed, wmin=1, wmax=16)
    if idx == 3:
        return road_knn(200_000 if small else 24_000_000, 2, seed)
    if idx == 4:
        if small:
            return rmat(16, 32, seed)
        return rmat(26, 32, seed)
    if idx == 5:
        if small:
            return batched_planted(64, seed, nmax=20_000)
        return batched_planted(4096, seed)
    raise ValueError("workload %r" % idx)


def describe(idx: int, small: bool = False) -> str:
    return NAMES[idx] + ("-small" if small else "")

"""Write tests/golden/workloads.json: the oracle's results on the full workloads.

Usage:  python tests/golden/make_golden.py 1 2 3 [4] [5]

Only graphgen (inputs) and oracle/ (the CPU reference) are called.  For each
workload it records the graph's size and content hash (so a generator mismatch
is told apart from an algorithm mismatch), the sweep count, the changed-vertex
count of every sweep, the community count before and after the split, the
modularity and an xxh3-128 hash of the final labels.  For a batch the labels of
each graph are computed separately and hashed in order.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np
import xxhash

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402
from graphgen import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")


def graph_hash(g) -> str:
    h = xxhash.xxh3_128()
    h.update(np.ascontiguousarray(g.offsets).view(np.uint8))
    h.update(np.ascontiguousarray(g.cols).view(np.uint8))
    if g.weights is not None:
        h.update(np.ascontiguousarray(g.weights).view(np.uint8))
    return h.hexdigest()


def labels_hash(labels) -> str:
    return xxhash.xxh3_128(np.ascontiguousarray(labels, dtype=np.int32).view(np.uint8)).hexdigest()


def run_single(idx: int) -> dict:
    t0 = time.time()
    g = workloads.make(idx)
    tg = time.time() - t0
    print("workload %d: n=%d nnz=%d generated in %.1fs" % (idx, g.n, g.nnz, tg), flush=True)
    t0 = time.time()
    raw = oracle.lpa(g, workloads.MAX_ITERS, workloads.TOLERANCE, split=False)
    t1 = time.time()
    out = oracle.split_bfs(g, raw.labels)
    t2 = time.time()
    q = oracle.modularity(g, out)
    rec = {
        "name": workloads.NAMES[idx], "n": g.n, "nnz": g.nnz, "graph_xxh128": graph_hash(g),
        "max_iters": workloads.MAX_ITERS, "tolerance": workloads.TOLERANCE,
        "iterations": int(raw.iterations), "dn": [int(x) for x in raw.dn],
        "processed": [int(x) for x in raw.processed],
        "communities_before_split": int(len(np.unique(raw.labels))),
        "communities": int(len(np.unique(out))),
        "modularity": q, "labels_xxh128": labels_hash(out),
        "raw_labels_xxh128": labels_hash(raw.labels),
        "oracle_seconds": {"sweeps": t1 - t0, "split": t2 - t1}, "oracle_threads": 1,
    }
    print(json.dumps(rec), flush=True)
    return rec


def run_batch(idx: int) -> dict:
    from concurrent.futures import ProcessPoolExecutor
    g = workloads.make(idx)
    G = g.num_graphs
    print("workload %d: %d graphs, n=%d nnz=%d" % (idx, G, g.n, g.nnz), flush=True)
    t0 = time.time()
    # Workers are forked after the batch exists, so they share its arrays
    # instead of each generating a copy.
    _BATCH[idx] = g
    with ProcessPoolExecutor(max_workers=os.cpu_count()) as ex:
        res = list(ex.map(_batch_one, [(idx, b) for b in range(G)], chunksize=8))
    h = xxhash.xxh3_128()
    iters = []
    for lab, it in res:
        h.update(lab.view(np.uint8))
        iters.append(it)
    rec = {"name": workloads.NAMES[idx], "n": g.n, "nnz": g.nnz, "graphs": G,
           "graph_xxh128": graph_hash(g), "max_iters": workloads.MAX_ITERS,
           "tolerance": workloads.TOLERANCE, "labels_xxh128": h.hexdigest(),
           "iterations": iters, "oracle_seconds_all_cores": time.time() - t0}
    print(json.dumps({k: v for k, v in rec.items() if k != "iterations"}), flush=True)
    return rec


_BATCH = {}


def _batch_one(arg):
    idx, b = arg
    if idx not in _BATCH:
        _BATCH[idx] = workloads.make(idx)
    sub = _BATCH[idx].subgraph(b)
    r = oracle.lpa(sub, workloads.MAX_ITERS, workloads.TOLERANCE)
    return r.labels, int(r.iterations)


def main(argv):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for a in argv:
        idx = int(a)
        rec = run_batch(idx) if idx == 5 else run_single(idx)
        data[str(idx)] = rec
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["1", "2", "3"])

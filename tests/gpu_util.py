"""Helpers for GPU tests: move graphgen graphs to the device, hash labels."""
from __future__ import annotations

import numpy as np
import torch
import xxhash


def to_device(g, dev="cuda", weights="as-is"):
    """(offsets, cols, weights) device tensors.  weights: "as-is" (None for
    unit-weight graphs), "ones" (materialise unit weights), "none"."""
    off = torch.from_numpy(np.ascontiguousarray(g.offsets, dtype=np.int64)).to(dev)
    cols = torch.from_numpy(np.ascontiguousarray(g.cols, dtype=np.int32)).to(dev)
    w = None
    if weights == "ones":
        w = torch.ones(g.nnz, dtype=torch.int32, device=dev)
    elif weights == "as-is" and g.weights is not None:
        w = torch.from_numpy(np.ascontiguousarray(g.weights, dtype=np.uint32).view(np.int32)).to(dev)
    return off, cols, w


def labels_hash(labels) -> str:
    if isinstance(labels, torch.Tensor):
        labels = labels.cpu().numpy()
    return xxhash.xxh3_128(np.ascontiguousarray(labels, dtype=np.int32).view(np.uint8)).hexdigest()


def graph_hash(g) -> str:
    h = xxhash.xxh3_128()
    h.update(np.ascontiguousarray(g.offsets).view(np.uint8))
    h.update(np.ascontiguousarray(g.cols).view(np.uint8))
    if g.weights is not None:
        h.update(np.ascontiguousarray(g.weights).view(np.uint8))
    return h.hexdigest()


def say(*args):
    print(*args, flush=True)

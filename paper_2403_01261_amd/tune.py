"""Autotuner for the degree tiers: degree bounds and sweep kernel variants.

The launch plan buckets vertices by degree into seven levels (plus degree 0
and hubs); each level runs one sweep kernel variant (lanes per vertex,
entries per lane, LDS table size, workgroup size).  Which bounds and variants
are fastest depends on the degree distribution and on the device, and never
on the result: every configuration gives the same labels.

tune() runs a coordinate descent over the levels: for each level it tries the
bounds {b/2, b, 2b} that keep the bounds non-decreasing, with every variant
that can hold rows of that length (and holds at most four times as many),
timing the production path (median wall time of a few runs of the workload:
gsl_lpa calls on probe graphs, or any callable, such as a batched call) and
keeping a change only when it is faster by more than the noise margin.  Two
passes, from each of two starting tables (the defaults, whose first level
runs a thread per vertex up to degree 32, and a finer one that starts a
level at degree 8), and the faster result wins: one level moved at a time
cannot shift every level up or down at once.  Results are cached as JSON per
device (and library version and probe), so later runs just load them:
load_or_tune().
"""
from __future__ import annotations

import json
import os
import statistics
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

Levels = List[Tuple[int, int]]

DEFAULT_LEVELS: Levels = [(32, 16), (64, 6), (128, 8), (512, 9), (1024, 17), (2048, 11), (4096, 13)]
FINE_LEVELS: Levels = [(8, 0), (32, 16), (64, 6), (128, 8), (512, 9), (2048, 11), (4096, 13)]
STARTS: List[Levels] = [DEFAULT_LEVELS, FINE_LEVELS]


def cache_path() -> str:
    return os.environ.get("GSL_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "gsl_lpa",
                                                            "tiers.json")


def valid(levels: Levels, variants: Sequence[dict]) -> bool:
    prev = 0
    for k, (b, v) in enumerate(levels):
        if not (0 <= v < len(variants)):
            return False
        if b < prev or b > variants[v]["capacity"]:
            return False
        prev = b
    return True


def options(levels: Levels, k: int, variants: Sequence[dict]) -> List[Tuple[int, int]]:
    """Candidate (bound, variant) pairs for level k with the others fixed."""
    b0 = levels[k][0]
    lo = levels[k - 1][0] if k > 0 else 0
    hi = levels[k + 1][0] if k + 1 < len(levels) else max(v["capacity"] for v in variants)
    bounds = sorted({b for b in (b0 // 2, b0, b0 * 2) if lo <= b <= hi})
    out = []
    for b in bounds:
        for v, info in enumerate(variants):
            if info["capacity"] < b or info["capacity"] > 4 * max(b, 8):
                continue
            out.append((b, v))
    return out


def search(measure: Callable[[Levels], float], variants: Sequence[dict], start: Optional[Levels] = None,
           passes: int = 2, margin: float = 0.02, log: Optional[Callable[[str], None]] = None) -> dict:
    """Coordinate descent; measure(levels) returns a time (lower is better)."""
    best = list(start or DEFAULT_LEVELS)
    if not valid(best, variants):
        raise ValueError("start levels are not valid for these variants")
    base = measure(best)
    best_t = base
    evals = 1
    for p in range(passes):
        changed = False
        for k in range(len(best)):
            for cand in options(best, k, variants):
                if cand == best[k]:
                    continue
                trial = best[:k] + [cand] + best[k + 1:]
                if not valid(trial, variants):
                    continue
                t = measure(trial)
                evals += 1
                if t < best_t * (1.0 - margin):
                    if log:
                        log("level %d: %s -> %s  %.3f -> %.3f ms" % (k, best[k], cand, best_t, t))
                    best, best_t, changed = trial, t, True
        if not changed:
            break
    return {"levels": [list(x) for x in best], "ms": best_t, "default_ms": base, "evaluations": evals}


def device_key(probe: str) -> str:
    import torch

    from . import gsl_version
    # architecture, compute units and memory size (the marketing name can be
    # empty, e.g. under a profiler)
    p = torch.cuda.get_device_properties(0)
    return "%s|%dcu|%dMiB|%s|%s" % (getattr(p, "gcnArchName", "") or p.name, p.multi_processor_count,
                                     p.total_memory >> 20, gsl_version(), probe)


def _read_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _write_cache(data: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_levels(run: Callable[[], None], levels: Levels, reps: int = 5) -> float:
    """Median wall time (ms) of run() under the given tiers, after one
    untimed run (which also builds the loop graph)."""
    import torch

    from . import gsl_set_tiers
    gsl_set_tiers(levels)
    run()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    return statistics.median(ts)


def graphs_runner(graphs, max_iters: int = 20, tol: float = 0.05) -> Callable[[], None]:
    """run() over probe graphs: list of (offsets, cols, weights, out) tensors,
    one gsl_lpa call each."""
    from . import gsl_lpa_ex

    def run():
        for off, cols, w, out in graphs:
            gsl_lpa_ex(off, cols, w, max_iters, tol, out=out)
    return run


def tune(run, probe: str, reps: int = 5, passes: int = 2, log=None) -> dict:
    """Tunes the tiers for run() (a callable doing one unit of the workload
    on the device, or a list of probe graphs, see graphs_runner), applies the
    result and caches it under `probe`."""
    from . import gsl_set_tiers, gsl_tier_variants
    if not callable(run):
        run = graphs_runner(run)
    variants = gsl_tier_variants()
    res = None
    evals = 0
    for start in STARTS:
        r = search(lambda lv: time_levels(run, lv, reps), variants, start=start, passes=passes, log=log)
        evals += r["evaluations"]
        if res is None:
            res = r
        elif r["ms"] < res["ms"]:
            res = dict(r, default_ms=res["default_ms"])
    res["evaluations"] = evals
    gsl_set_tiers([tuple(x) for x in res["levels"]])
    res["when"] = time.strftime("%Y-%m-%dT%H:%M:%S")
    data = _read_cache()
    data[device_key(probe)] = res
    _write_cache(data)
    return res


def load_or_tune(run, probe: str, retune: bool = False, **kw) -> dict:
    """Applies the cached tiers for this device and probe, tuning first if
    there are none (or retune)."""
    from . import gsl_set_tiers, gsl_tier_variants
    if not retune:
        rec = _read_cache().get(device_key(probe))
        if rec and valid([tuple(x) for x in rec["levels"]], gsl_tier_variants()):
            gsl_set_tiers([tuple(x) for x in rec["levels"]])
            rec = dict(rec)
            rec["cached"] = True
            return rec
    return tune(run, probe, **kw)

"""Benchmark: GSL-LPA (label-propagation sweeps + split) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 2]

A step is one full gsl_lpa call (degree plan, synchronous sweeps with pruning
until dN/N <= 0.05 or 20 sweeps, split) on a graph already resident in HBM.
value = |E| / time per step, |E| = directed CSR entries (every undirected edge
twice, as the paper counts edges after adding reverse edges).  The timed steps
run the production path (the sweep loop as captured graphs, no per-launch
events).

Extra objects on the JSON line:
  roofline      the dominant sweep kernel: algorithmic bytes per launch over
                its average launch time, from HIP events recorded around every
                launch on the library's stream in a second pass of the same
                number of steps right after the timed ones (same kernels and
                launch shapes; events inside the timed steps would add gaps
                to them), against the 8 TB/s HBM peak; traffic = measured HBM
                bytes per launch from rocprofv3 counters (profiles/traffic.json),
                null when absent or stale.
  cpu_baseline  the CPU oracle (single thread, untuned) timed on this host.
  gather_reference
                a plain PyTorch gather of an int32 label array by the
                workload's column array (the sweeps' bound), beside the
                sweep phase's row entries per second (phases).
  tiers         the degree tiers the timed runs used: by default the tier
                autotuner (paper_2403_01261_amd/tune.py) runs first on the
                same workload, outside every timed region.

--workload 5 measures the batch of 4,096 planted graphs instead: graphs/s of
the plain per-graph loop (one gsl_lpa call per graph), of one gsl_lpa_batched
call, and of the continuous-batching server against a plain one-graph-per-call
server on the same Poisson stream (2,000 requests/s), with p50/p99 latency;
every path's labels are checked to be identical.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD_TEXT = {
    1: "planted partition: 10,000 vertices, 100 blocks of 100, intra prob 0.1, ~2 inter edges "
       "per vertex, unit weights",
    2: "R-MAT scale 22 (4,194,304 vertices), edge factor 16, a/b/c/d 0.57/0.19/0.19/0.05, "
       "symmetrised, no self loops or duplicates, uint32 weights uniform in [1,16]",
    3: "road-like 2-D random geometric graph, 24M vertices, union-symmetrised 2 nearest "
       "neighbours, unit weights",
    4: "web-scale R-MAT scale 26 (67,108,864 vertices), edge factor 32, a/b/c/d "
       "0.57/0.19/0.19/0.05, symmetrised, unit weights",
    5: "batch of 4,096 planted-partition graphs, N log-uniform in [200, 200,000], 5-500 blocks, "
       "mean degree U[8, 32] with 2 inter-block, unit weights",
}
NUM_TIERS = 9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tier_bytes(t: dict, weighted: bool) -> int:
    """Algorithmic bytes a sweep kernel moves for one tier, summed over its
    launches: per listed vertex the 4 B list entry (+1 B active flag in sparse
    launches that scan the tier; a launch that walks a frontier reads 4 B per
    frontier entry instead); per processed vertex two 8 B offsets and its own
    4 B label; per row entry a 4 B column, a 4 B gathered label (+4 B weight);
    per changed vertex its 4 B new label and 1 B change flag; 1 B per
    neighbour flag set."""
    scans = t["launches"] - t.get("frontier_launches", 0)
    listed = t["vertices"] * scans + t.get("frontier_listed", 0)
    return (listed * 4 + t["vertices"] * t["sparse_launches"] * 1
            + t["processed"] * (16 + 4)
            + t["edges"] * (8 + (4 if weighted else 0))
            + t["changed"] * 5 + t["marked"] * 1)


def _code_only(text: str) -> str:
    """C++/HIP source without comments and with whitespace runs collapsed, so
    that editing a comment does not count as a change of the kernels."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(csrc: str = None) -> str:
    """Hash of the kernel sources' code (the measured traffic in
    profiles/traffic.json is reported only while it matches)."""
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2403_01261_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str, levels, launches_per_step: int, path: str = None):
    """Measured HBM bytes per launch of `kernel`: the profiled bytes per
    gsl_lpa call (all dispatches of the kernel in a run of known call count)
    over the launches one call makes.  None unless the record was taken with
    the same kernel code and the same tier table as the timed run."""
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path) or launches_per_step <= 0:
        return None
    with open(path) as f:
        rec = json.load(f)
    entry = rec.get(workload, {}).get(kernel)
    if not entry or entry.get("source_hash") != source_hash():
        return None
    if [list(x) for x in entry.get("levels", [])] != [list(x) for x in levels]:
        return None
    if "bytes_per_step" not in entry:
        return None
    return int(round(entry["bytes_per_step"] / launches_per_step))


COPY_BYTES = 1 << 30  # plain device-to-device copy used to calibrate the PMC counters


# L2-to-memory requests by size: read bytes are 32, 64 and 128 times these
# counts, write bytes 64 times the 64-byte writes and 32 times the rest.
RAW_READ = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")
RAW_WRITE = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum")


def _dispatch_bytes(d: str, kind: str):
    """{dispatch_id: (kernel_name, bytes)} of L2-to-memory traffic from a
    rocprofv3 --pmc csv directory (kind "read" or "write"): from the request
    counts by size when the run collected them, else from FETCH_SIZE /
    WRITE_SIZE (KiB).  Returns (record, source)."""
    names = RAW_READ if kind == "read" else RAW_WRITE
    raw = {c: _read_counter_csv(d, c) for c in names}
    if all(raw.values()):
        out = {}
        for did, (name, _) in raw[names[0]].items():
            v = {c: raw[c].get(did, (name, 0.0))[1] for c in names}
            if kind == "read":
                b = 32.0 * v[names[0]] + 64.0 * v[names[1]] + 128.0 * v[names[2]]
            else:
                b = 32.0 * (v[names[0]] - v[names[1]]) + 64.0 * v[names[1]]
            out[did] = (name, b)
        return out, "request counts " + ", ".join(names)
    counter = "FETCH_SIZE" if kind == "read" else "WRITE_SIZE"
    rec = _read_counter_csv(d, counter)
    return {k: (n, v * 1024.0) for k, (n, v) in rec.items()}, counter


def _read_counter_csv(d: str, counter: str):
    """{dispatch_id: (kernel_name, value)} from a rocprofv3 --pmc csv directory."""
    import csv
    import glob
    out = {}
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(path) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                did = int(r["Dispatch_Id"])
                name, val = r["Kernel_Name"], float(r["Counter_Value"])
                prev = out.get(did)
                out[did] = (name, val + (prev[1] if prev else 0.0))
    return out


def _kernel_stats(d: str):
    """Per kernel from a rocprofv3 kernel trace: all dispatches, and those
    that did work.  A sweep kernel enqueued after its loop has converged
    returns at once; dispatches shorter than 5% of the kernel's longest are
    counted as such empty launches."""
    import csv
    import glob
    paths = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
    if not paths:
        return []
    per = {}
    with open(paths[0]) as f:
        for r in csv.DictReader(f):
            dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            per.setdefault(r["Kernel_Name"], []).append(dt)
    total = sum(sum(v) for v in per.values()) or 1
    rows = []
    for name, ds in per.items():
        cut = 0.05 * max(ds)
        work = [x for x in ds if x >= cut]
        rows.append({"Name": name, "Calls": len(ds), "WorkCalls": len(work),
                     "WorkAvgNs": sum(work) / len(work), "TotalDurationNs": sum(ds),
                     "Percentage": 100.0 * sum(ds) / total})
    rows.sort(key=lambda r: -r["TotalDurationNs"])
    return rows


def _short(name: str) -> str:
    return name.replace("gsl::(anonymous namespace)::", "").replace("void ", "")


def summarize_pmc(fetch_dir: str, write_dir: str, trace_dir: str, workload: int, kernel: str,
                  commands: list, calls: int, levels, launches_per_call: int, out_dir: str = None,
                  trace_calls: int = 0) -> dict:
    """Traffic of `kernel` from two counter runs (reads, then writes): the
    sum over every dispatch of the kernel divided by the number of gsl_lpa
    calls the run made (`calls`, each with `launches_per_call` working
    launches of the kernel under the tier table `levels`).  Launches enqueued
    after a loop converged return at once and add next to nothing, so bytes
    per call over working launches per call is the traffic of one working
    launch -- the same launch set the benchmark's per-launch durations
    average over.  With the request counts by size the bytes are exact and
    the plain COPY_BYTES copy of the runs checks them; with FETCH_SIZE /
    WRITE_SIZE they are scaled by what those read for the copy.  Writes
    traffic.json and the kernel-trace summary into out_dir (profiles/)."""
    from graphgen import workloads
    fetch, fsrc = _dispatch_bytes(fetch_dir, "read")
    write, wsrc = _dispatch_bytes(write_dir, "write")

    def calib(rec):
        copies = [v for n, v in rec.values() if "copyBuffer" in n]
        return max(copies) if copies else None

    cf, cw = calib(fetch), calib(write)
    kf = [v for n, v in fetch.values() if _short(n).startswith(kernel)]
    kw = [v for n, v in write.values() if _short(n).startswith(kernel)]
    if not kf or not kw or not cf or not cw:
        raise SystemExit("counter runs lack the kernel %r or the calibration copy" % kernel)
    exact_r, exact_w = fsrc.startswith("request"), wsrc.startswith("request")
    sf = 1.0 if exact_r else COPY_BYTES / cf
    sw = 1.0 if exact_w else COPY_BYTES / cw
    fetch_step = sum(kf) * sf / calls
    write_step = sum(kw) * sw / calls
    fetch_b = fetch_step / launches_per_call
    write_b = write_step / launches_per_call
    wname = workloads.NAMES[workload]
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    path = os.path.join(out_dir, "traffic.json")
    rec = {}
    if os.path.exists(path):
        with open(path) as f:
            rec = json.load(f)
    rec.setdefault(wname, {})[kernel] = {
        "bytes_per_step": int(round(fetch_step + write_step)), "calls": calls,
        "launches_per_call": launches_per_call, "levels": [list(x) for x in levels],
        "bytes_per_launch": int(round(fetch_b + write_b)), "fetch_bytes_per_launch": int(round(fetch_b)),
        "write_bytes_per_launch": int(round(write_b)), "dispatches": len(kf),
        "read_counters": fsrc, "write_counters": wsrc,
        "copy_read_bytes": cf, "copy_write_bytes": cw, "copy_bytes": COPY_BYTES, "scale_fetch": sf,
        "scale_write": sw, "source_hash": source_hash(), "commands": commands}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
        f.write("\n")
    # Short text summary of the kernel trace next to it.
    stats = _kernel_stats(trace_dir)
    tag = kernel.replace("<", "-").replace(">", "").replace(", ", "-")
    md = os.path.join(out_dir, "%s_%s.md" % (wname, tag))
    with open(md, "w") as f:
        f.write("# %s on %s\n\n" % (kernel, wname))
        f.write("Commands (repository root, MI355X):\n\n")
        for c in commands:
            f.write("    %s\n" % c)
        f.write("\nTier table (max degree, variant) of the runs: %s.\n\n" % json.dumps([list(x) for x in levels]))
        f.write("L2-to-memory traffic of `%s`: %d dispatches over %d gsl_lpa calls of %d working launches "
                "each; per working launch read %.3f GB, write %.3f GB.  Reads from %s, writes from %s, summed "
                "over the dispatches; the plain %d MiB copy of the same runs reads %.1f MiB and writes %.1f MiB "
                "by the same counters (scale applied: x%.4f / x%.4f).\n\n"
                % (kernel, len(kf), calls, launches_per_call, fetch_b / 1e9, write_b / 1e9, fsrc, wsrc,
                   COPY_BYTES >> 20, cf / 2 ** 20, cw / 2 ** 20, sf, sw))
        mine = [r for r in stats if _short(r["Name"]).startswith(kernel)] if stats else []
        if mine and trace_calls > 0:
            tot = sum(r["TotalDurationNs"] for r in mine) / 1e6
            f.write("Launches as the benchmark counts them (its `launches_per_step`): %d per gsl_lpa call.  "
                    "The trace's %d calls spend %.2f ms in `%s`: %.3f ms per call, %.3f ms per launch (for the "
                    "kernel the benchmark's roofline names, the figure its `avg_launch_ms` measures with HIP "
                    "events).\n\n"
                    % (launches_per_call, trace_calls, tot, kernel, tot / trace_calls,
                       tot / (trace_calls * launches_per_call)))
        if stats:
            f.write("Kernel trace of the first command.  `calls` counts every dispatch; sweep kernels "
                    "enqueued after the loop converged return at once, so `working calls` and their "
                    "average count only dispatches of at least 5% of the kernel's longest.\n\n")
            f.write("| kernel | calls | working calls | avg us (working) | total ms | % |\n"
                    "|---|---|---|---|---|---|\n")
            for r in stats[:24]:
                f.write("| %s | %d | %d | %.1f | %.2f | %.1f |\n" % (
                    _short(r["Name"])[:72], r["Calls"], r["WorkCalls"], r["WorkAvgNs"] / 1e3,
                    r["TotalDurationNs"] / 1e6, r["Percentage"]))
    return rec[wname][kernel]


def calibration_copy():
    """A plain device copy of COPY_BYTES, the reference the traffic counters
    are scaled by."""
    import torch
    src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def gather_reference(cols, n, reps=5):
    """Random 4-byte gathers as a plain PyTorch kernel does them: an int32
    array of n labels indexed by the workload's own column array (original
    vertex order), timed with events on torch's stream.  The sweeps are bound
    by such gathers (one per row entry), not by streaming bandwidth."""
    import torch
    lab = torch.arange(n, dtype=torch.int32, device=cols.device)
    out = torch.empty_like(cols)
    torch.index_select(lab, 0, cols, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.index_select(lab, 0, cols, out=out)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del lab, out
    return {"gathers_per_s": cols.numel() / (ms / 1000.0), "ms": round(ms, 3),
            "method": "torch.index_select of an int32 array of n labels by the column array "
                      "(original vertex order), %d runs" % reps}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def pinned_runs(fn, budget_s: float, max_runs: int):
    """Runs fn() on one core (the calling thread pinned, as taskset does)
    until max_runs runs or the time budget is spent (at least one run).
    Returns (list of seconds, last result, core)."""
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    times, res = [], None
    try:
        t_all = time.perf_counter()
        while len(times) < max_runs and (not times or time.perf_counter() - t_all + times[-1] <= budget_s):
            t0 = time.perf_counter()
            res = fn()
            times.append(time.perf_counter() - t0)
    finally:
        os.sched_setaffinity(0, old)
    return times, res, core


def cpu_baseline(g, max_iters, tol, w32=None, what="the whole workload", budget_s=25.0, max_runs=5):
    """The oracle (single thread, untuned, pinned to one core), as many full
    GSL-LPA runs (sweeps + split) of graph g as fit the budget, at most
    max_runs; median and mean."""
    import statistics

    import oracle
    fn = (lambda: oracle.lpa(g, max_iters, tol)) if w32 is None else (lambda: oracle.lpa_f32(g, w32, max_iters, tol))
    times, r, core = pinned_runs(fn, budget_s, max_runs)
    med, mean = statistics.median(times), statistics.mean(times)
    return {"value": g.nnz / med, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": "%d full oracle GSL-LPA run(s) (sweeps + split) of %s, single thread pinned to core %d; "
                      "median %.2f s, mean %.2f s" % (len(times), what, core, med, mean),
            "runs": len(times), "seconds_median": round(med, 3), "seconds_mean": round(mean, 3),
            "value_mean": g.nnz / mean, "iterations": int(r.iterations),
            "host": {"nproc": os.cpu_count(), "cpu": cpu_model()}}, r


def golden_record(idx: int):
    """Expected values the oracle wrote for workload idx (tests/golden)."""
    path = os.path.join(ROOT, "tests", "golden", "workloads.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(str(idx))


def labels_hash(t) -> str:
    import numpy as np
    import xxhash
    return xxhash.xxh3_128(np.ascontiguousarray(t.cpu().numpy(), dtype=np.int32).view(np.uint8)).hexdigest()


# Workloads too large for a bounded oracle run: the oracle runs on a smaller
# graph of the same recipe instead (name, generator arguments).
CPU_SAMPLE = {4: ("R-MAT scale 21, edge factor 32, same a/b/c/d, relabelling and seed as rmat-s26, unit weights",
                  dict(scale=21, edge_factor=32))}


def run_tuner(args, run, probe):
    """Degree tiers for the timed runs: the autotuner's choice for this
    workload (tuning time is outside every timed region), or the defaults."""
    import paper_2403_01261_amd as gsl
    if args.tiers == "default":
        gsl.gsl_set_tiers(None)
        return {"source": "default", "levels": gsl.gsl_get_tiers()}
    from paper_2403_01261_amd import tune
    t0 = time.time()
    log("tier autotuner: key %r, cache %s" % (tune.device_key(probe), tune.cache_path()))
    res = tune.load_or_tune(run, probe, retune=args.tiers == "tune", reps=3, passes=2, log=log)
    log("tiers tuned in %.1fs: %.3f ms -> %.3f ms, %s" % (time.time() - t0, res["default_ms"], res["ms"],
                                                          res["levels"]))
    return {"source": "autotuner (cached)" if res.get("cached") else "autotuner", "levels": res["levels"],
            "probe": probe,
            "probe_ms_default": round(res["default_ms"], 3), "probe_ms_tuned": round(res["ms"], 3),
            "evaluations": res["evaluations"], "seconds": round(time.time() - t0, 1)}


def roofline_from_stats(stats, weighted, steps, wname, n):
    """Dominant sweep kernel over a list of timing-mode stats dicts."""
    ms_tier = [sum(st["tiers"][t]["ms"] for st in stats) for t in range(NUM_TIERS)]
    dom = max(range(1, NUM_TIERS), key=lambda t: ms_tier[t])
    agg = {key: sum(st["tiers"][dom][key] for st in stats)
           for key in ("vertices", "launches", "processed", "edges", "changed", "marked",
                       "sparse_launches", "frontier_launches", "frontier_listed")}
    agg["vertices"] = stats[0]["tiers"][dom]["vertices"]
    launches = agg["launches"]
    bytes_total = tier_bytes(agg, weighted)
    avg_ms = ms_tier[dom] / max(launches, 1)
    achieved = bytes_total / max(launches, 1) / (avg_ms / 1000.0) / 1e9 if avg_ms > 0 else 0.0
    import paper_2403_01261_amd as gsl
    variants = gsl.gsl_tier_variants()
    levels = gsl.gsl_get_tiers()
    kernel = "hub_insert" if dom == NUM_TIERS - 1 else gsl.variant_kernel_name(variants[levels[dom - 1][1]], weighted, n)
    lps = launches // max(steps, 1)
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(wname, kernel, levels, lps),
            "kernel": kernel, "tier": dom, "launches_per_step": launches // max(steps, 1),
            "avg_launch_ms": round(avg_ms, 4),
            "algorithmic_bytes_per_launch": bytes_total // max(launches, 1)}


# The continuous server's session for the batch of 4,096 graphs: room for a
# little over half of the batch at once (64 Mi vertices, 1.6 G entries), up
# to sixteen sweeps per step.  A step ends anyway once every resident graph
# has stopped, so long steps cost a quiet server nothing and spare a busy one
# the per-step plan, copies and synchronisations (p50 at 2,000 / 5,000 /
# 20,000 requests/s: 1.6 / 3.4 / 47 ms with 16 sweeps, 3.3 / 8.4 / 45 ms
# with 4).
SESSION_CAP = (64 << 20, 1600 << 20, 4096)
SESSION_SWEEPS = 16

_POOL_BATCH = None


def _pool_one(k):
    import oracle
    from graphgen import workloads
    r = oracle.lpa(_POOL_BATCH.subgraph(k), workloads.MAX_ITERS, workloads.TOLERANCE)
    return r.labels


def batched_cpu_pool(b):
    """The oracle on every graph of the batch, in a process pool over all the
    host's cores (graphs are independent).  The workers are forked, so this
    runs before anything touches the GPU."""
    import concurrent.futures
    import multiprocessing

    import xxhash
    global _POOL_BATCH
    _POOL_BATCH = b
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    with concurrent.futures.ProcessPoolExecutor(max_workers=cores,
                                                mp_context=multiprocessing.get_context("fork")) as ex:
        res = list(ex.map(_pool_one, range(b.num_graphs), chunksize=8))
    dt = time.perf_counter() - t0
    _POOL_BATCH = None
    h = xxhash.xxh3_128()
    for lab in res:
        h.update(lab.view("uint8"))
    gold = golden_record(5)
    return {"value": b.num_graphs / dt, "unit": "graphs/s", "cores": cores, "kind": "oracle",
            "sample": "all %d graphs, one oracle GSL-LPA run each, in a pool of %d worker processes, %.1f s"
                      % (b.num_graphs, cores, dt),
            "edges_per_s": b.nnz / dt, "labels_xxh128": h.hexdigest(),
            "labels_match_oracle_golden": bool(gold and gold.get("labels_xxh128") == h.hexdigest()),
            "host": {"nproc": os.cpu_count(), "cpu": cpu_model()}}


def batched_cpu_sample(b, seconds=15.0):
    """The oracle, one thread pinned to one core, on the batch's graphs in
    order until the time budget is spent."""
    import oracle
    from graphgen import workloads
    old = os.sched_getaffinity(0)
    core = min(old)
    os.sched_setaffinity(0, {core})
    done, edges, labels = 0, 0, []
    try:
        ts = time.perf_counter()
        while done < b.num_graphs and time.perf_counter() - ts < seconds:
            sub = b.subgraph(done)
            labels.append(oracle.lpa(sub, workloads.MAX_ITERS, workloads.TOLERANCE).labels)
            edges += sub.nnz
            done += 1
        dt = time.perf_counter() - ts
    finally:
        os.sched_setaffinity(0, old)
    return {"value": done / dt, "unit": "graphs/s", "cores": 1, "kind": "oracle",
            "sample": "the first %d of the %d graphs (%d entries), one oracle GSL-LPA run each, single thread "
                      "pinned to core %d, %.1f s" % (done, b.num_graphs, edges, core, dt),
            "edges_per_s": edges / dt, "host": {"nproc": os.cpu_count(), "cpu": cpu_model()}}, labels


def batched_gpu(b, args, tiers_mode):
    """The batch of planted graphs on the GPU, resident in HBM: the plain
    per-graph loop (one gsl_lpa call per graph), one gsl_lpa_batched call,
    and request streams through the two servers (slot batches of
    gsl_lpa_graphs calls; sweep-level continuous batching on a gsl_session)
    and through a plain one-graph-per-call server, at 2,000 requests/s and
    above what the plain path can serve.  Every path's labels are compared."""
    import numpy as np
    import torch

    import paper_2403_01261_amd as gsl
    from graphgen import workloads
    from paper_2403_01261_amd.serve import (ContinuousServer, GpuExecutor, PlainExecutor, Request, Server,
                                            SessionBackend, poisson_arrivals, summarize)
    dev = torch.device("cuda:0")
    G, N, nnz = b.num_graphs, b.n, b.nnz
    mi, tol = workloads.MAX_ITERS, workloads.TOLERANCE
    vb, eb = b.vtx_base, b.edge_base
    off = torch.from_numpy(b.offsets).to(dev)
    cols = torch.from_numpy(b.cols).to(dev)
    vb_d = torch.from_numpy(vb).to(dev)
    eb_d = torch.from_numpy(eb).to(dev)
    loc_off = [torch.from_numpy(b.offsets[vb[k]:vb[k + 1] + 1] - eb[k]).to(dev) for k in range(G)]
    loc_cols = [cols[eb[k]:eb[k + 1]] for k in range(G)]
    out_plain = torch.empty(N, dtype=torch.int32, device=dev)
    out_batch = torch.empty(N, dtype=torch.int32, device=dev)
    views = [out_plain[vb[k]:vb[k + 1]] for k in range(G)]
    torch.cuda.synchronize()

    def plain_loop(count):
        for k in range(count):
            gsl.gsl_lpa_ex(loc_off[k], loc_cols[k], None, mi, tol, out=views[k])

    # tiers: tuned on the batched call over a prefix of the batch, or the defaults
    P = min(G, 512)
    vb_p, eb_p = vb_d[:P + 1], eb_d[:P + 1]
    off_p, cols_p = off[:vb[P] + 1], cols[:eb[P]]
    out_p = out_batch[:vb[P]]
    targs = argparse.Namespace(**vars(args))
    targs.tiers = tiers_mode
    tiers = run_tuner(targs, lambda: gsl.gsl_lpa_batched(vb_p, eb_p, off_p, cols_p, None, mi, tol, out=out_p),
                      "%s prefix %d" % (workloads.describe(5, args.small), P))
    steps = max(1, args.batched_steps)
    for k in range(2):
        gsl.gsl_lpa_batched(vb_d, eb_d, off, cols, None, mi, tol, out=out_batch)
        plain_loop(min(G, 64))
    torch.cuda.synchronize()
    ts = time.perf_counter()
    plain_loop(G)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - ts
    log("plain loop: %.3f s, %.1f graphs/s" % (plain_s, G / plain_s))
    ts = time.perf_counter()
    for k in range(steps):
        gsl.gsl_lpa_batched(vb_d, eb_d, off, cols, None, mi, tol, out=out_batch)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - ts) / steps
    log("batched: %.3f s/call, %.1f graphs/s" % (batch_s, G / batch_s))
    _, iters_b, st_b = gsl.gsl_lpa_batched(vb_d, eb_d, off, cols, None, mi, tol, out=out_batch, timing=True)
    gold = golden_record(5)
    hb = labels_hash(out_batch)
    same_plain_batch = bool(torch.equal(out_plain, out_batch))
    res = {"graphs": G, "n": N, "nnz": nnz, "tiers": tiers,
           "batched": {"graphs_per_s": round(G / batch_s, 1), "edges_per_s": nnz / batch_s,
                       "ms": round(1000.0 * batch_s, 3), "calls_timed": steps,
                       "iterations_max": st_b["iterations"], "iterations_mean": round(float(iters_b.float().mean()), 2),
                       "ms_plan": round(st_b["ms_plan"], 3), "ms_sweeps": round(st_b["ms_sweeps"], 3),
                       "ms_split": round(st_b["ms_split"], 3)},
           "plain": {"graphs_per_s": round(G / plain_s, 1), "edges_per_s": nnz / plain_s,
                     "ms": round(1000.0 * plain_s, 3)},
           "speedup_batched_vs_plain": round(plain_s / batch_s, 2),
           "labels_identical_plain_batched": same_plain_batch,
           "labels_match_oracle_golden": bool(gold and gold.get("labels_xxh128") == hb),
           "roofline": roofline_from_stats([st_b], False, 1, workloads.NAMES[5], N)}
    # request streams
    served = {}
    streams = [("continuous", 2000.0), ("continuous", 5000.0), ("continuous", 20000.0),
               ("slots", 2000.0), ("slots", 5000.0), ("slots", 20000.0), ("plain", 2000.0)]
    for mode, rate in streams:
        times = poisson_arrivals(G, rate, 240301261)
        if mode == "plain":
            ex = PlainExecutor(mi, tol)
            reqs = [Request(rid=k, arrival=float(times[k]), n=int(vb[k + 1] - vb[k]), nnz=int(eb[k + 1] - eb[k]),
                            payload=(loc_off[k], loc_cols[k], None)) for k in range(G)]
            srv = Server(ex, slots=1, budget_bytes=64 << 30, max_batch_graphs=1)
        elif mode == "slots":
            ex = GpuExecutor(2, mi, tol)
            reqs = [Request(rid=k, arrival=float(times[k]), n=int(vb[k + 1] - vb[k]), nnz=int(eb[k + 1] - eb[k]),
                            payload=(off[vb[k]:vb[k + 1] + 1], cols, None)) for k in range(G)]
            srv = Server(ex, slots=2, budget_bytes=64 << 30)
        else:
            ex = SessionBackend(max_vertices=SESSION_CAP[0], max_entries=SESSION_CAP[1], max_graphs=SESSION_CAP[2],
                                max_iters=mi, tolerance=tol)
            reqs = [Request(rid=k, arrival=float(times[k]), n=int(vb[k + 1] - vb[k]), nnz=int(eb[k + 1] - eb[k]),
                            payload=(loc_off[k], loc_cols[k], None)) for k in range(G)]
            srv = ContinuousServer(ex, sweeps_per_step=SESSION_SWEEPS)
        torch.cuda.synchronize()
        srv.serve(reqs)
        if mode != "plain":
            ex.close()
        summ = summarize(reqs, getattr(srv, "batches", None))
        summ["labels_identical_to_plain"] = all(r.state == "done" and torch.equal(r.labels, views[r.rid])
                                                for r in reqs)
        if mode == "continuous":
            summ["steps"] = srv.steps
            summ["session_bytes"] = gsl.Session.device_bytes(*SESSION_CAP)
            summ["session_capacity"] = {"vertices": SESSION_CAP[0], "entries": SESSION_CAP[1],
                                        "graphs": SESSION_CAP[2], "sweeps_per_step": SESSION_SWEEPS}
        key = "%s_%d" % (mode, int(rate))
        served[key] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
        log("served %s: %s" % (key, served[key]))
        del reqs
    res["served"] = served
    del off, cols, loc_off, loc_cols, out_plain, out_batch, views
    torch.cuda.synchronize()
    return res


def batched_profile(b, calls: int) -> int:
    """Exactly `calls` gsl_lpa_batched calls over the whole batch with the
    default tiers (as the batch rides along in the default run), then one in
    timing mode for the launch counts (a profiler sees calls + 1 calls)."""
    import torch

    import paper_2403_01261_amd as gsl
    from graphgen import workloads
    gsl.load()
    dev = torch.device("cuda:0")
    off = torch.from_numpy(b.offsets).to(dev)
    cols = torch.from_numpy(b.cols).to(dev)
    vb = torch.from_numpy(b.vtx_base).to(dev)
    eb = torch.from_numpy(b.edge_base).to(dev)
    out = torch.empty(b.n, dtype=torch.int32, device=dev)
    mi, tol = workloads.MAX_ITERS, workloads.TOLERANCE
    for _ in range(calls):
        gsl.gsl_lpa_batched(vb, eb, off, cols, None, mi, tol, out=out)
    torch.cuda.synchronize()
    _, _, st = gsl.gsl_lpa_batched(vb, eb, off, cols, None, mi, tol, out=out, timing=True)
    print(json.dumps({"profile_calls": calls + 1, "levels": gsl.gsl_get_tiers(),
                      "tier_launches": [t["launches"] for t in st["tiers"]],
                      "ms_tier": [round(t["ms"], 4) for t in st["tiers"]],
                      "iterations": st["iterations"]}), flush=True)
    return 0


def bench_batched(args):
    """Workload 5 as the headline: graphs/s of one gsl_lpa_batched call over
    the 4,096 graphs, with the plain loop, the servers and the CPU baselines
    beside it."""
    from graphgen import workloads
    t0 = time.time()
    b = workloads.make(5, small=args.small)
    log("generated batch: %d graphs, N=%d, nnz=%d in %.1fs" % (b.num_graphs, b.n, b.nnz, time.time() - t0))
    if args.profile_steps:
        return batched_profile(b, args.profile_steps)
    pool = None if args.no_cpu_baseline or args.small else batched_cpu_pool(b)
    import paper_2403_01261_amd as gsl
    gsl.load()
    res = batched_gpu(b, args, args.tiers)
    cpu = None
    if not args.no_cpu_baseline:
        cpu, labels = batched_cpu_sample(b)
    G = b.num_graphs
    batch_s = res["batched"]["ms"] / 1000.0
    line = {"metric": "graphs/s, batched (one gsl_lpa_batched call) vs plain per-graph gsl_lpa calls",
            "value": G / batch_s, "unit": "graphs/s", "n_gpus": 1, "steps": res["batched"]["calls_timed"],
            "warmup": 2, "ms_per_step": 1000.0 * batch_s, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "%s: %s" % (workloads.describe(5, args.small),
                                                "small variant: 64 planted graphs, N log-uniform in "
                                                "[200, 20,000]" if args.small else WORKLOAD_TEXT[5]),
                       "graphs": G, "n": b.n, "nnz": b.nnz, "max_iters": workloads.MAX_ITERS,
                       "tolerance": workloads.TOLERANCE, "weights": "NULL (unit)"},
            "roofline": res.pop("roofline"), "cpu_baseline": cpu, "cpu_all_cores": pool}
    line.update(res)
    print(json.dumps(line), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=4, choices=sorted(WORKLOAD_TEXT),
                    help="1 planted-10k, 2 rmat-s22, 3 road-24m, 4 rmat-s26 (default: the largest graph), "
                         "5 batched-4096")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small", action="store_true", help="the small variant of the workload (quick checks)")
    ap.add_argument("--tiers", choices=("tune", "cached", "default"), default=None,
                    help="degree tiers of the timed runs: run the tier autotuner first, reuse its "
                         "cached result for this device and workload (tuning only if there is none), or "
                         "keep the library defaults (the default for rmat-s26, whose tuning takes minutes; "
                         "the others tune)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="run exactly this many production gsl_lpa calls after generation and exit "
                         "(for rocprofv3 counter and trace runs; prints the tier table and launches per call)")
    ap.add_argument("--weights-f32", action="store_true",
                    help="pass the workload's weights as fp32 values (summed in fp64, gsl_lpa_f32)")
    ap.add_argument("--split-techniques", action="store_true",
                    help="also time the split techniques (union-find, LP, LP with pruning) on the raw LPA labels")
    ap.add_argument("--batched-steps", type=int, default=3,
                    help="gsl_lpa_batched calls timed for the batch of 4,096 graphs")
    ap.add_argument("--no-batched", action="store_true",
                    help="rmat-s26: leave out the batch of 4,096 graphs (plain, batched and served paths)")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="run a plain 1 GiB device copy first (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "TRACE_DIR"),
                    help="write profiles/traffic.json from rocprofv3 counter runs and exit")
    ap.add_argument("--kernel", default=None, help="kernel for --summarize-pmc")
    ap.add_argument("--commands", nargs="*", default=[], help="commands recorded by --summarize-pmc")
    ap.add_argument("--calls", type=int, default=0, help="gsl_lpa calls of the profiled runs (--summarize-pmc)")
    ap.add_argument("--levels", default=None, help="tier table of the profiled runs, JSON (--summarize-pmc)")
    ap.add_argument("--launches-per-call", type=int, default=0,
                    help="working launches of the kernel per call (--summarize-pmc)")
    ap.add_argument("--trace-calls", type=int, default=0,
                    help="gsl_lpa calls of the kernel-trace run (--summarize-pmc)")
    args = ap.parse_args(argv)
    if args.tiers is None:
        args.tiers = "default" if args.workload == 4 else "tune"
    if args.summarize_pmc:
        r = summarize_pmc(*args.summarize_pmc, args.workload, args.kernel, args.commands, args.calls,
                          json.loads(args.levels), args.launches_per_call, trace_calls=args.trace_calls)
        print(json.dumps(r))
        return 0
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2
    if args.pmc_copy:
        calibration_copy()
    if args.workload == 5:
        return bench_batched(args)

    # The batch of 4,096 graphs rides along with rmat-s26: generated, and its
    # all-cores CPU baseline run (forked workers), before anything touches the
    # GPU.
    b5, pool5 = None, None
    if args.workload == 4 and not (args.no_batched or args.small or args.profile_steps):
        from graphgen import workloads as _w
        t0 = time.time()
        b5 = _w.make(5)
        log("generated batched-4096: %d graphs, nnz=%d in %.1fs" % (b5.num_graphs, b5.nnz, time.time() - t0))
        if not args.no_cpu_baseline:
            pool5 = batched_cpu_pool(b5)
            log("oracle process pool: %.1f graphs/s on %d cores, labels match golden: %s"
                % (pool5["value"], pool5["cores"], pool5["labels_match_oracle_golden"]))

    import numpy as np
    import torch

    import graphgen
    import paper_2403_01261_amd as gsl
    from graphgen import workloads

    gsl.load()
    dev = torch.device("cuda:0")
    t0 = time.time()
    g = workloads.make(args.workload, small=args.small)
    log("generated %s: n=%d nnz=%d in %.1fs" % (workloads.NAMES[args.workload], g.n, g.nnz,
                                                 time.time() - t0))
    weighted = g.weights is not None or args.weights_f32
    off = torch.from_numpy(g.offsets).to(dev)
    cols = torch.from_numpy(g.cols).to(dev)
    if args.weights_f32:
        wsrc = g.weights if g.weights is not None else np.ones(g.nnz, dtype=np.uint32)
        w = torch.from_numpy(wsrc.astype(np.float32)).to(dev)
    else:
        w = torch.from_numpy(g.weights.view(np.int32)).to(dev) if g.weights is not None else None
    lpa_call = gsl.gsl_lpa_f32 if args.weights_f32 else gsl.gsl_lpa_ex
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    mi, tol = workloads.MAX_ITERS, workloads.TOLERANCE
    torch.cuda.synchronize()

    tiers = (run_tuner(args, lambda: lpa_call(off, cols, w, mi, tol, out=labels),
                       workloads.describe(args.workload, args.small))
             if not args.weights_f32 else {"source": "default (fp32 weights use the default tiers)"})
    if args.profile_steps:
        # exactly profile_steps production calls, then the launch counts the
        # traffic summary needs (from one more call in timing mode, after the
        # profiled ones: rocprofv3 sees profile_steps + 1 calls)
        for k in range(args.profile_steps):
            lpa_call(off, cols, w, mi, tol, out=labels)
        torch.cuda.synchronize()
        _, st = lpa_call(off, cols, w, mi, tol, timing=True, out=labels)
        print(json.dumps({"profile_calls": args.profile_steps + 1, "levels": gsl.gsl_get_tiers(),
                          "tier_launches": [t["launches"] for t in st["tiers"]],
                          "ms_tier": [round(t["ms"], 4) for t in st["tiers"]],
                          "iterations": st["iterations"]}), flush=True)
        return 0
    for k in range(args.warmup):
        lpa_call(off, cols, w, mi, tol, out=labels)
        log("warmup %d done" % k)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        lpa_call(off, cols, w, mi, tol, out=labels)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1000.0 * elapsed / max(args.steps, 1)
    value = g.nnz * args.steps / elapsed
    log("timed %d steps: %.3f ms/step, %.3g edges/s" % (args.steps, ms_per_step, value))
    stats = []
    for k in range(args.steps):
        _, st = lpa_call(off, cols, w, mi, tol, timing=True, out=labels)
        stats.append(st)
    log("event pass: %.3f ms/step with per-launch events" % (sum(s["ms_total"] for s in stats) / len(stats)))

    # Dominant sweep kernel over the event pass.
    wname = workloads.NAMES[args.workload]
    roofline = roofline_from_stats(stats, weighted, args.steps, wname, g.n)
    # Whole sweep phase (all tier kernels + apply) for context.
    sweep_ms = sum(st["ms_sweeps"] for st in stats) / len(stats)
    sweep_bytes = sum(tier_bytes(dict(st["tiers"][t], vertices=st["tiers"][t]["vertices"]), weighted)
                      for st in stats for t in range(1, NUM_TIERS)) / len(stats)
    last = stats[-1]
    sweep_entries = sum(st["tiers"][t]["edges"] for st in stats for t in range(1, NUM_TIERS)) / len(stats)
    phases = {"ms_plan": round(sum(s["ms_plan"] for s in stats) / len(stats), 3),
              "ms_sweeps": round(sweep_ms, 3),
              "ms_split": round(sum(s["ms_split"] for s in stats) / len(stats), 3),
              "sweep_phase_GBps": round(sweep_bytes / (sweep_ms / 1000.0) / 1e9, 1) if sweep_ms else None,
              "sweep_entries_per_s": sweep_entries / (sweep_ms / 1000.0) if sweep_ms else None,
              "ms_reorder": round(sum(s["ms_reorder"] for s in stats) / len(stats), 3),
              "renumbered": last["renumbered"],
              "ms_per_step_with_events": round(sum(s["ms_total"] for s in stats) / len(stats), 3),
              "iterations": last["iterations"], "changed": last["changed"]}

    split_cmp = None
    if args.split_techniques:
        raw, _ = lpa_call(off, cols, w, mi, tol, split=False)
        split_cmp = {}
        ref = None
        for tech in ("union-find", "lp", "lpp"):
            out, rounds, ms = gsl.gsl_split_ex(off, cols, raw, tech)
            same = True if ref is None else bool(torch.equal(out, ref))
            ref = out if ref is None else ref
            split_cmp[tech] = {"ms": round(ms, 3), "rounds": rounds, "same_labels": same}
            log("split %s: %.3f ms, %d rounds" % (tech, ms, rounds))

    gref = gather_reference(cols, g.n)
    log("gather reference: %.3g gathers/s (sweep phase: %.3g row entries/s)" % (gref["gathers_per_s"],
                                                                           phases["sweep_entries_per_s"] or 0))

    # the timed labels against the oracle's expected values (tests/golden)
    gold = golden_record(args.workload) if not (args.small or args.weights_f32) else None
    parity = None
    if gold is not None and gold.get("nnz") == g.nnz:
        h = labels_hash(labels)
        parity = {"labels_xxh128": h, "labels_match_oracle_golden": h == gold["labels_xxh128"],
                  "iterations_match": last["iterations"] == gold["iterations"],
                  "dn_match": list(last["changed"]) == list(gold["dn"])}
        log("labels vs the oracle's golden hash: %s" % parity)

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        if args.workload in CPU_SAMPLE and not args.small:
            # a smaller graph of the same recipe; the GPU labels of that
            # graph are checked against the oracle's as well
            what, kw = CPU_SAMPLE[args.workload]
            sg = graphgen.rmat(kw["scale"], kw["edge_factor"], workloads.SEED_BASE + args.workload)
            cpu, ref = cpu_baseline(sg, mi, tol, None, what="a %d-entry sample graph (%s)" % (sg.nnz, what))
            so = torch.from_numpy(sg.offsets).to(dev)
            sc = torch.from_numpy(sg.cols).to(dev)
            slab, _ = lpa_call(so, sc, None, mi, tol)
            cpu["labels_match_gpu"] = bool(np.array_equal(slab.cpu().numpy(), ref.labels))
            cpu["sample_graph"] = {"n": sg.n, "nnz": sg.nnz}
            if gold is not None and "oracle_seconds" in gold:
                osec = gold["oracle_seconds"]
                cpu["full_workload_reference"] = {
                    "edges_per_s": g.nnz / (osec["sweeps"] + osec["split"]),
                    "note": "one unpinned single-thread oracle run of the whole workload when the golden file "
                            "was written (another host: context only)"}
            del so, sc, slab
        else:
            cpu, ref = cpu_baseline(g, mi, tol, w.cpu().numpy() if args.weights_f32 else None,
                                    max_runs=1 if args.workload == 3 else 5)
            got = labels.cpu().numpy()
            cpu["labels_match_gpu"] = bool(np.array_equal(got, ref.labels))
        log("oracle: %.3g edges/s, labels match: %s" % (cpu["value"], cpu["labels_match_gpu"]))

    batched = None
    if b5 is not None:
        # free the large graph first
        del off, cols, w, labels
        torch.cuda.synchronize()
        gsl.gsl_release()
        torch.cuda.empty_cache()
        batched = batched_gpu(b5, args, "default")
        if not args.no_cpu_baseline:
            batched["cpu_baseline"], _ = batched_cpu_sample(b5)
        batched["cpu_all_cores"] = pool5
        batched["workload"] = "%s: %s" % (workloads.NAMES[5], WORKLOAD_TEXT[5])

    line = {"metric": "edges/s (|E|/time) on 1 MI355X + % HBM peak", "value": value,
            "unit": "edges/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64" if args.weights_f32 else "u32", "data": "synthetic",
            "config": {"workload": "%s: %s" % (wname, WORKLOAD_TEXT[args.workload]), "n": g.n,
                       "nnz": g.nnz, "max_iters": mi, "tolerance": tol,
                       "weights": ("fp32 array, fp64 sums" if args.weights_f32 else
                                   "uint32 array" if weighted else "NULL (unit)")},
            "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "phases": phases,
            "gather_reference": gref, "tiers": tiers,
            "split_techniques": split_cmp, "batched_served": batched,
            "context": "paper: 844M edges/s, sk-2005 3.8B edges, 2x Xeon Gold 6226R, 64 threads"}
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

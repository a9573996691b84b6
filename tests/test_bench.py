"""bench.py's measurement logic on the CPU: the algorithmic bytes of a tier,
the working-launch cut of a kernel trace, and the traffic summary scaled by
the calibration copy (synthetic rocprofv3 CSV files)."""
import csv
import json
import os

import bench


def test_tier_bytes_per_unit():
    zero = {"vertices": 0, "launches": 0, "sparse_launches": 0, "processed": 0, "edges": 0, "changed": 0,
            "marked": 0}

    def one(**kw):
        t = dict(zero)
        t.update(kw)
        return t

    assert bench.tier_bytes(one(vertices=1, launches=1), False) == 4          # list entry
    assert bench.tier_bytes(one(vertices=1, sparse_launches=1), False) == 1   # active flag
    assert bench.tier_bytes(one(processed=1), False) == 20                    # two offsets + own label
    assert bench.tier_bytes(one(edges=1), False) == 8                         # column + gathered label
    assert bench.tier_bytes(one(edges=1), True) == 12                         # + weight
    assert bench.tier_bytes(one(changed=1), False) == 5                       # new label + change flag
    assert bench.tier_bytes(one(marked=1), False) == 1                        # neighbour flag
    # a tier listed in 3 launches, one of them sparse
    t = one(vertices=10, launches=3, sparse_launches=1, processed=25, edges=100, changed=7, marked=40)
    assert bench.tier_bytes(t, True) == 10 * 3 * 4 + 10 + 25 * 20 + 100 * 12 + 7 * 5 + 40
    # two more launches walked frontiers of 3 and 2 vertices: 4 B per entry,
    # no scan of the tier list and no flag reads
    t = one(vertices=10, launches=5, sparse_launches=1, frontier_launches=2, frontier_listed=5)
    assert bench.tier_bytes(t, False) == 10 * 3 * 4 + 10 + 5 * 4


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def test_kernel_stats_counts_working_launches(tmp_path):
    rows = [["k<1>(args)", 0, 100_000], ["k<1>(args)", 200_000, 300_000], ["k<1>(args)", 400_000, 402_000],
            ["other()", 500_000, 501_000]]
    _write(str(tmp_path / "t" / "x_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    stats = {r["Name"]: r for r in bench._kernel_stats(str(tmp_path / "t"))}
    k = stats["k<1>(args)"]
    assert k["Calls"] == 3 and k["WorkCalls"] == 2 and k["WorkAvgNs"] == 100_000
    assert abs(sum(r["Percentage"] for r in stats.values()) - 100.0) < 1e-9


def test_summarize_pmc_scales_by_the_copy(tmp_path):
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    copy = "__amd_rocclr_copyBuffer"
    kern = "void gsl::(anonymous namespace)::sweep_lds<8, 5, 256, 2>(gsl::SweepArgs)"
    # the copy of 1 GiB reads as 0.5 GiB in FETCH_SIZE (scale 2) and 1 GiB in
    # WRITE_SIZE (scale 1); two calls of two working launches each, plus an
    # empty launch after convergence
    _write(str(tmp_path / "f" / "f_counter_collection.csv"), hdr,
           [[1, copy, "FETCH_SIZE", 524288.0], [2, kern, "FETCH_SIZE", 1000.0], [3, kern, "FETCH_SIZE", 3000.0],
            [4, kern, "FETCH_SIZE", 10.0], [5, kern, "FETCH_SIZE", 1000.0], [6, kern, "FETCH_SIZE", 3000.0]])
    _write(str(tmp_path / "w" / "w_counter_collection.csv"), hdr,
           [[1, copy, "WRITE_SIZE", 1048576.0], [2, kern, "WRITE_SIZE", 100.0], [3, kern, "WRITE_SIZE", 300.0],
            [4, kern, "WRITE_SIZE", 0.0], [5, kern, "WRITE_SIZE", 100.0], [6, kern, "WRITE_SIZE", 300.0]])
    out = tmp_path / "profiles"
    levels = [[32, 16], [64, 6], [128, 8], [512, 9], [1024, 17], [2048, 11], [4096, 13]]
    rec = bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "t"), 2,
                              "sweep_lds<8, 5, 256, 2>", ["cmd"], 2, levels, 2, out_dir=str(out))
    assert rec["dispatches"] == 5 and rec["calls"] == 2 and rec["launches_per_call"] == 2
    assert rec["scale_fetch"] == 2.0 and rec["scale_write"] == 1.0
    assert rec["fetch_bytes_per_launch"] == round(8010 * 1024 * 2 / 4)
    assert rec["write_bytes_per_launch"] == 800 * 1024 // 4
    assert rec["bytes_per_step"] == (8010 * 2 + 800) * 1024 // 2
    saved = json.load(open(out / "traffic.json"))
    entry = saved["rmat-s22"]["sweep_lds<8, 5, 256, 2>"]
    assert entry["source_hash"] == bench.source_hash() and entry["levels"] == levels
    assert (out / "rmat-s22_sweep_lds-8-5-256-2.md").exists()
    # the benchmark reports the traffic only for the same tier table
    path = str(out / "traffic.json")
    got = bench.measured_traffic("rmat-s22", "sweep_lds<8, 5, 256, 2>", levels, 2, path=path)
    assert got == round(entry["bytes_per_step"] / 2)
    other = [list(x) for x in levels]
    other[0][0] = 8
    assert bench.measured_traffic("rmat-s22", "sweep_lds<8, 5, 256, 2>", other, 2, path=path) is None
    assert bench.measured_traffic("rmat-s22", "sweep_lds<8, 5, 256, 2>", levels, 0, path=path) is None
    assert bench.measured_traffic("rmat-s26", "sweep_lds<8, 5, 256, 2>", levels, 2, path=path) is None


def test_summarize_pmc_from_request_counts(tmp_path):
    """With the L2 request counts by size the bytes are exact (no scaling):
    32 / 64 / 128 bytes per read request, 64 per 64-byte write, 32 per other
    write; the copy is recorded as a check."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    copy = "__amd_rocclr_copyBuffer"
    kern = "gsl::(anonymous namespace)::hub_insert(gsl::SweepArgs, gsl::(anonymous namespace)::HubArgs)"
    r32, r64, r128 = bench.RAW_READ
    wall, w64 = bench.RAW_WRITE
    reads = [[1, copy, r32, 0], [1, copy, r64, 0], [1, copy, r128, (1 << 30) // 128]]
    writes = [[1, copy, wall, (1 << 30) // 64], [1, copy, w64, (1 << 30) // 64]]
    for d in (2, 3):  # two working launches in one call
        reads += [[d, kern, r32, 10], [d, kern, r64, 100], [d, kern, r128, 1000]]
        writes += [[d, kern, wall, 50], [d, kern, w64, 20]]
    _write(str(tmp_path / "r" / "r_counter_collection.csv"), hdr, reads)
    _write(str(tmp_path / "w" / "w_counter_collection.csv"), hdr, writes)
    out = tmp_path / "profiles"
    levels = [[32, 16], [64, 6], [128, 8], [512, 9], [1024, 17], [2048, 11], [4096, 13]]
    rec = bench.summarize_pmc(str(tmp_path / "r"), str(tmp_path / "w"), str(tmp_path / "t"), 4, "hub_insert",
                              ["cmd"], 1, levels, 2, out_dir=str(out))
    assert rec["scale_fetch"] == 1.0 and rec["scale_write"] == 1.0
    assert rec["copy_read_bytes"] == 1 << 30 and rec["copy_write_bytes"] == 1 << 30
    assert rec["fetch_bytes_per_launch"] == 32 * 10 + 64 * 100 + 128 * 1000
    assert rec["write_bytes_per_launch"] == 32 * 30 + 64 * 20
    assert rec["read_counters"].startswith("request counts")

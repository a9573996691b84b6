"""The tier autotuner's search and cache logic on the CPU (a synthetic cost
stands in for timing the device)."""
import json

import numpy as np

from paper_2403_01261_amd import tune

# The library's variant menu (gsl_tier_variant), as capacities and groups.
VARIANTS = [{"group": g, "per_lane": k, "capacity": g * k} for g, k in
            [(1, 8), (8, 2), (4, 4), (16, 2), (8, 4), (32, 2), (16, 4), (64, 2), (32, 4), (64, 8), (128, 4),
             (256, 8), (512, 4), (512, 8), (1024, 8), (1, 16), (1, 32), (256, 4), (1, 64)]]


def test_defaults_are_valid_and_options_respect_bounds():
    assert tune.valid(tune.DEFAULT_LEVELS, VARIANTS)
    bad = list(tune.DEFAULT_LEVELS)
    bad[2] = (200, 3)  # capacity 32
    assert not tune.valid(bad, VARIANTS)
    bad = list(tune.DEFAULT_LEVELS)
    bad[3] = (20, 5)  # below level 2's bound
    assert not tune.valid(bad, VARIANTS)
    bad = list(tune.DEFAULT_LEVELS)
    bad[1] = (64, 99)  # no such variant
    assert not tune.valid(bad, VARIANTS)
    ok = list(tune.DEFAULT_LEVELS)
    ok[1] = (64, 6)  # a group variant, and a thread variant on a later level
    ok[2] = (64, 16)
    assert not tune.valid(ok, VARIANTS)  # thread<32> cannot hold degree 64
    ok[2] = (128, 8)
    assert tune.valid(ok, VARIANTS)
    assert tune.valid(tune.FINE_LEVELS, VARIANTS)
    for start in tune.STARTS:
        for k in range(7):
            opts = tune.options(start, k, VARIANTS)
            assert opts
            for b, v in opts:
                assert b <= VARIANTS[v]["capacity"] <= 4 * max(b, 8)


def test_search_finds_the_cheaper_configuration():
    # synthetic cost: variant 7 is cheaper than 8 at level 2, and a level-3
    # bound of 256 with variant 9 beats 512/9; everything else neutral
    def cost(levels):
        c = 10.0
        if levels[2][1] == 7:
            c -= 1.0
        if tuple(levels[3]) == (256, 9):
            c -= 2.0
        return c

    seen = []
    res = tune.search(lambda lv: (seen.append(list(lv)), cost(lv))[1], VARIANTS)
    assert res["default_ms"] == 10.0
    assert res["ms"] == 7.0
    assert res["levels"][2][1] == 7 and tuple(res["levels"][3]) == (256, 9)
    assert all(tune.valid(lv, VARIANTS) for lv in seen)
    assert res["evaluations"] == len(seen)


def test_search_keeps_defaults_within_noise():
    rng = np.random.default_rng(1)
    res = tune.search(lambda lv: 10.0 + rng.uniform(-0.05, 0.05), VARIANTS, margin=0.02)
    assert [tuple(x) for x in res["levels"]] == tune.DEFAULT_LEVELS


def test_cache_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("GSL_TUNE_CACHE", str(tmp_path / "sub" / "tiers.json"))
    assert tune._read_cache() == {}
    tune._write_cache({"dev|probe": {"levels": [[8, 0]] * 7}})
    with open(tmp_path / "sub" / "tiers.json") as f:
        assert json.load(f)["dev|probe"]["levels"][0] == [8, 0]
    assert tune._read_cache()["dev|probe"]["levels"][0] == [8, 0]

"""Timing mode (gsl_stats): the per-sweep, per-tier and phase times add up,
every sweep that ran has its own time (also when the renumbering copy ran
sweep 0), and timing changes no result."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from graphgen import workloads  # noqa: E402
from tests.gpu_util import say, to_device  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_01261_amd as m
    m.load()
    return m


@pytest.mark.parametrize("layout", ["original", "renumbered"])
def test_timing_stats_add_up(gsl, layout):
    g = workloads.make(2, small=True)
    off, cols, w = to_device(g)
    ref, st0 = gsl.gsl_lpa_ex(off, cols, w, layout=layout)
    lab, st = gsl.gsl_lpa_ex(off, cols, w, layout=layout, timing=True)
    torch.cuda.synchronize()
    assert torch.equal(lab, ref) and st["iterations"] == st0["iterations"]
    it = st["iterations"]
    folded = st["renumbered"] and st["processed"][0] == g.n - st["tiers"][0]["vertices"] and st["ms_sweep"][0] == 0
    first = 1 if folded else 0
    say(layout, "iterations", it, "folded", folded, "ms_sweep", [round(x, 3) for x in st["ms_sweep"]],
        "ms_sweeps", round(st["ms_sweeps"], 3))
    assert it >= 3
    if layout == "renumbered":
        assert folded  # the rows of this workload are strictly increasing
    assert all(x > 0 for x in st["ms_sweep"][first:it])
    # the sweep phase also holds the empty launches enqueued after the loop
    # stopped, so the sweeps that ran take at most all of it
    total = sum(st["ms_sweep"])
    assert total <= st["ms_sweeps"] * 1.02 + 0.01
    tiers = sum(t["ms"] for t in st["tiers"]) + st["ms_hub_finish"]
    assert tiers <= total * 1.02 + 0.01
    for t in st["tiers"][1:]:
        if t["vertices"]:
            assert t["launches"] == it - first
    assert st["ms_plan"] <= st["ms_total"] and st["ms_sweeps"] <= st["ms_total"]

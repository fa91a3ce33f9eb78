"""Host-side logic of bench.py that needs no GPU: the oracle sample behind the paper workload's
cpu_baseline.  Run in full, it covers every T gate of the circuits it names.  Given a budget, it
starts no gate once the budget is spent, so it counts a prefix of the gates and says so in
`sample`."""
import re

import bench


def test_paper_baseline_in_full_counts_every_gate():
    out = bench.paper_cpu_baseline([("paper_d2_n12", 4, None), ("paper_d3_n12", 4, 6)])
    assert out["kind"] == "oracle" and out["unit"] == "non-Clifford gates/s"
    # N layers for the first circuit, 6 for the second, one T gate per layer
    assert "(10 gates," in out["sample"]
    assert "paper_d2_n12 n=4 in full" in out["sample"]
    assert "paper_d3_n12 n=4 layers=6 in full" in out["sample"]
    assert out["value"] > 0.0


def test_paper_baseline_budget_stops_before_the_next_gate():
    # a budget spent before the first gate: no gate starts in either circuit
    out = bench.paper_cpu_baseline([("paper_d2_n12", 4, 8), ("paper_d3_n12", 4, 8)], budget=0.0)
    assert re.findall(r"first (\d+) of (\d+)", out["sample"]) == [("0", "8"), ("0", "8")]
    assert "(0 gates," in out["sample"] and out["value"] == 0.0
    # a budget that is never reached runs everything
    out = bench.paper_cpu_baseline([("paper_d2_n12", 4, 8)], budget=1e9)
    assert "paper_d2_n12 n=4 layers=8 in full (8 gates," in out["sample"]

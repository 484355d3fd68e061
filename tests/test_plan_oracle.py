"""Pins of the MapDevice oracle (Algorithm 2, Eq. 7-9) against the paper's
printed Table II and against closed-form decision thresholds."""
import math
import os

import pytest

from oracle import plan

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table2_base_costs.txt")
NAMES = {"Aggregation (Hash)": plan.AGG, "Filtering": plan.FILTER, "Shuffling": plan.SHUFFLE,
         "Projection": plan.PROJECT, "Join (Hash)": plan.JOIN, "Expand": plan.EXPAND,
         "Scan (CSV File)": plan.SCAN, "Sorting": plan.SORT}


def golden_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, pref, cost = [x.strip() for x in line.rsplit(",", 2)]
        rows.append((name, pref, float(cost)))
    return rows


def test_table2_matches_paper():
    rows = golden_rows()
    assert len(rows) == 8
    for name, pref, cost in rows:
        assert plan.TABLE2[NAMES[name]] == (pref, cost)
    assert plan.BASE_TRANS0 == 0.1
    assert plan.INFPT0 == 150 * 1024


@pytest.mark.parametrize("b", [1.0, 0.9, 0.8])
def test_single_op_threshold_closed_form(b):
    # a lone operation is both first and last: Trans goes to GPU, so CPU wins iff
    # b/x + 0.1 x > b x, i.e. x < sqrt(b / (b - 0.1))
    xstar = math.sqrt(b / (b - 0.1))
    for x, dev in [(xstar * 0.999, plan.CPU), (xstar * 1.001, plan.GPU), (0.01, plan.CPU), (100.0, plan.GPU)]:
        devs, _ = plan.map_device([b], batch_bytes=x * plan.INFPT0 * 12, num_cores=12)
        assert devs == [dev], (b, x)


def test_chain_is_all_cpu_below_first_threshold_and_all_gpu_above():
    # With Table II bases every first operation needs x > sqrt(b / (b - 0.1)) >= 1.054 to reach the GPU,
    # and an operation after a CPU one faces the same threshold, so a chain is entirely on the CPU below
    # the smallest such threshold (1.0541 for b = 1.0, 1.0607 for 0.9, 1.0690 for 0.8 -> min 1.0541) and,
    # once x exceeds every threshold, entirely on the GPU.
    bases = [b for _, (_, b) in sorted(plan.TABLE2.items())]
    for x in (0.2, 0.6, 0.9, 1.0, 1.05):
        assert plan.map_device(bases, x * plan.INFPT0, 1)[0] == [plan.CPU] * len(bases), x
    for x in (1.07, 1.5, 10.0):
        assert plan.map_device(bases, x * plan.INFPT0, 1)[0] == [plan.GPU] * len(bases), x


def test_hand_traced_chains():
    # chain scan -> filter -> project -> agg with Table II bases (0.8, 1.0, 0.9, 1.0)
    bases = [0.8, 1.0, 0.9, 1.0]
    # x = 0.5: first op: CPU 0.4 vs GPU 1.6 + 0.05 -> CPU; filter (prev CPU): CPU 0.5 vs 2.0 + 0.05 -> CPU;
    # project: 0.45 vs 1.8 + 0.05 -> CPU; agg (last): 0.5 vs 2.05 -> CPU
    devs, costs = plan.map_device(bases, 0.5 * plan.INFPT0 * 4, 4)
    assert devs == [plan.CPU] * 4
    assert costs == pytest.approx([0.4, 0.5, 0.45, 0.5])
    # x = 2: first: CPU 1.6 vs GPU 0.4 + 0.2 -> GPU; filter (prev GPU, middle): CPU 2.0 + 0.2 vs 0.5 -> GPU;
    # project: 1.8 + 0.2 vs 0.45 -> GPU; agg (last): 2.0 vs 0.5 + 0.2 -> GPU
    devs, costs = plan.map_device(bases, 2.0 * plan.INFPT0 * 4, 4)
    assert devs == [plan.GPU] * 4
    assert costs == pytest.approx([0.6, 0.5, 0.45, 0.7])
    # x = 1.0: first: CPU 0.8 vs GPU 0.8 + 0.1 -> CPU; filter (prev CPU): 1.0 vs 1.0 + 0.1 -> CPU;
    # project (prev CPU): 0.9 vs 0.9 + 0.1 -> CPU; agg: 1.0 vs 1.1 -> CPU
    devs, _ = plan.map_device(bases, plan.INFPT0, 1)
    assert devs == [plan.CPU] * 4
    # x = 1.06: first (b = 0.8, threshold 1.069): CPU; filter (b = 1.0, prev CPU, threshold 1.0541): GPU;
    # project (b = 0.9, middle after GPU, threshold 0.9487): GPU; agg (last, threshold 1.0541): GPU
    devs, _ = plan.map_device(bases, 1.06 * plan.INFPT0, 1)
    assert devs == [plan.CPU, plan.GPU, plan.GPU, plan.GPU]


def test_tie_stays_on_gpu():
    # base 0.1 with x = 1 as a middle op after GPU: CPU = 0.1 + 0.1 = 0.2, GPU = 0.1 -> GPU; construct exact tie:
    # lone op, b = 0.2, x = sqrt(0.2/0.1) = sqrt 2: CPU = 0.2 sqrt2, GPU = 0.2/sqrt2 + 0.1 sqrt2 = 0.2 sqrt2
    x = math.sqrt(2.0)
    devs, _ = plan.map_device([0.2], x * plan.INFPT0, 1)
    cpu, gpu = 0.2 * x, 0.2 / x + 0.1 * x
    assert devs == [plan.GPU if not gpu > cpu else plan.CPU]

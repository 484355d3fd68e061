"""MapDevice oracle -- TEST INFRASTRUCTURE ONLY.

Algorithm 2 of the paper (Sec. III-D) with the device cost model of
Eq. 7-9, written out step by step in the paper's notation:

* Part = micro-batch bytes / NumCores (the per-core data partition, Sec. III-D);
* CPU_o = baseCost_o * Part / InfPT            (Eq. 7)
* GPU_o = baseCost_o * InfPT / Part            (Eq. 8)
* Trans_o = baseTransCost * Part / InfPT       (Eq. 9), baseTransCost = 0.1;
* every operation starts on the GPU; walking the chain from the first
  operation, Trans_o is added to GPU_o when o is the first or the last
  operation or operation o-1 runs on the CPU, and to CPU_o otherwise;
  o moves to the CPU when GPU_o > CPU_o (a tie stays on the GPU).

Base costs are Table II's; InfPT starts at 150 KB (Sec. III-D, read as
150 * 1024 bytes).
"""
from __future__ import annotations

AGG, FILTER, SHUFFLE, PROJECT, JOIN, EXPAND, SCAN, SORT = range(8)

# Table II: operation -> (initial preference, base cost).
TABLE2 = {
    AGG: ("CPU", 1.0),
    FILTER: ("CPU", 1.0),
    SHUFFLE: ("CPU", 1.0),
    PROJECT: ("Neutral", 0.9),
    JOIN: ("Neutral", 0.9),
    EXPAND: ("Neutral", 0.9),
    SCAN: ("GPU", 0.8),
    SORT: ("GPU", 0.8),
}

INFPT0 = 150.0 * 1024.0
BASE_TRANS0 = 0.1
CPU, GPU = 0, 1


def map_device(bases, batch_bytes, num_cores, infpt=INFPT0, base_trans=BASE_TRANS0):
    """Return (devices, costs) for the chain whose base costs are `bases`."""
    n = len(bases)
    part = batch_bytes / num_cores
    plan = [GPU] * n
    costs = [0.0] * n
    for o in range(n):
        cpu = bases[o] * (part / infpt)
        gpu = bases[o] * (infpt / part)
        trans = base_trans * (part / infpt)
        if o == 0 or o == n - 1 or plan[o - 1] == CPU:
            gpu += trans
        else:
            cpu += trans
        if gpu > cpu:
            plan[o] = CPU
        costs[o] = cpu if plan[o] == CPU else gpu
    return plan, costs

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


def splitmix64(state):
    """One step of SplitMix64 (Steele, Lea and Flood): returns (output, new state)."""
    m = (1 << 64) - 1
    state = (state + 0x9E3779B97F4A7C15) & m
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31), state


class InfPTRegression:
    """Eq. 10 (Sec. III-E): InfPT = b0 + b1 * Throughput + b2 * Latency, fitted
    by least squares on the recorded micro-batches (the last `history`, all if
    0) and evaluated at the target throughput (the largest seen) and the
    target latency (given, else the mean past MaxLat).  Reading (no value is
    printed for these): fewer than three records, collinear regressors or a
    non-positive prediction keep the previous InfPT; the returned value is
    multiplied by 1 + jitter * u with u uniform in [-1, 1] from SplitMix64 so
    the recorded InfPTs vary and the fit is identifiable."""

    def __init__(self, init_bytes=INFPT0, history=0, jitter=0.1, seed=0):
        self.cur = float(init_bytes)
        self.history = history
        self.jitter = jitter
        self.state = seed
        self.rec = []

    def record(self, infpt_used, thput, maxlat):
        self.rec.append((float(thput), float(maxlat), float(infpt_used)))

    def next(self, target_latency=0.0):
        import numpy as np
        rec = self.rec[-self.history:] if self.history else self.rec
        if len(rec) >= 3:
            x = np.array([[1.0, t, lat] for t, lat, _ in rec])
            y = np.array([v for _, _, v in rec])
            if np.linalg.matrix_rank(x, tol=1e-9 * np.abs(x).max()) == 3:
                beta = np.linalg.lstsq(x, y, rcond=None)[0]
                tmax = max(t for t, _, _ in self.rec)
                lat = target_latency if target_latency > 0 else float(np.mean([lat for _, lat, _ in self.rec]))
                pred = beta[0] + beta[1] * tmax + beta[2] * lat
                if np.isfinite(pred) and pred > 0:
                    self.cur = float(pred)
        out, self.state = splitmix64(self.state)
        u = (out >> 11) * 2.0 ** -53 * 2.0 - 1.0
        return self.cur * (1.0 + self.jitter * u)

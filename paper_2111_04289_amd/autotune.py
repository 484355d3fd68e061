"""Autotuner of the windowed group-by's tile and schedule parameters.

The parameters (``lms_tuning``: rows per scan chunk, target rows per hash
partition, rows per aggregation piece, persistent scan workgroups per CU, LDS
group-table slots per aggregation workgroup) trade parallelism and occupancy
against per-workgroup overhead and L2 locality; the best values depend on the
batch-size mix.  A candidate whose run reports a nonzero device status is
discarded.  ``tune`` searches them by coordinate descent on
a workload timed on the GPU (each coordinate swept with the others fixed, up
to two passes) and writes the winners per workload to JSON; ``apply`` loads them into
the library before a run.  Every candidate runs the same kernels, so results
do not depend on the tuning (the GPU tests check a non-default setting against
the oracle).

    python -m paper_2111_04289_amd.autotune --workload sliding batched --out tuned.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import lms

PACKAGED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")

SPACE = {
    "chunk_rows": [0, 2048, 8192, 32768, 65536],
    "lds_groups": [0, 1024],
    "part_rows": [0, 4096, 8192, 32768],
    "piece_rows": [0, 2048, 4096, 16384],
    "grid_per_cu": [0, 2, 5, 8],
}
# Coordinates of the descent.  Partition and piece sizes default to multiples of
# the LDS table size, so the table-size coordinate moves all three coherently;
# the others then refine.
COORDS = [("lds_groups",), ("chunk_rows",), ("part_rows",), ("piece_rows",), ("grid_per_cu",)]
DEFAULT = {k: 0 for k in SPACE}


def _values(coord):
    import itertools
    return list(itertools.product(*(SPACE[name] for name in coord)))


def apply(workload: str, path: str | None = None):
    """Loads the tuned parameters of ``workload`` (from ``path``, else the packaged
    file) into the library; returns them, or None (defaults) if there are none."""
    path = path or PACKAGED
    params = None
    if os.path.exists(path):
        with open(path) as f:
            params = json.load(f).get(workload, {}).get("params")
    if params:
        lms.set_tuning(**{k: int(params.get(k, 0)) for k in SPACE})
    else:
        lms.set_tuning()
    return params


def _sliding(torch, dev, rows):
    from . import datagen
    cols = [torch.from_numpy(c).to(dev) for c in datagen.config1(rows)]
    preds = [(2, lms.LT, datagen.CONFIG1_VAL_CUT)]
    aggs = [(lms.COUNT, 0), (lms.SUM, 2), (lms.MIN, 2), (lms.MAX, 2), (lms.AVG, 3)]
    w = lms.Window(0, 10000, 1000, 0)
    groups = lms.Groups(rows * 10, aggs, dev)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = lms.Workspace(dev)

    def run():
        lms.lms_window_agg(cols, 1, w, aggs, preds, groups=groups, d_count=cnt, workspace=ws)

    def ok():
        return int(cnt[1]) == 0

    return run, ok


def _batched(torch, dev, rows, nbatch=256, seed=11):
    from . import datagen
    cols = [torch.from_numpy(c).to(dev) for c in datagen.config1(rows)]
    rng = np.random.default_rng(seed)
    hi = min(8 << 20, rows)
    sizes = np.exp(rng.uniform(np.log(1024), np.log(hi), nbatch)).astype(np.int64)
    offs = [4 * int(rng.integers(0, (rows - s) // 4 + 1)) for s in sizes]  # 16-byte aligned, as separate buffers
    batches = [[c[o:o + int(s)] for c in cols] for o, s in zip(offs, sizes)]
    aggs = [(lms.COUNT, 0), (lms.SUM, 4)]
    job = lms.MultiJob(1, lms.Window(0, 1000, 0, 0), aggs, [(2, lms.LT, 500)], [(2, 2, 0)], device=dev)
    state = {}

    def run():
        if state.get("tuning") != lms.get_tuning():  # plans depend on the tuning
            job.prepare(batches, groups=state.get("groups"), d_counts=state.get("cnt"))
            state["groups"], state["cnt"] = job.groups, job.d_counts
            state["tuning"] = lms.get_tuning()
        job.launch()

    def ok():
        return not bool(state["cnt"][:, 1].any())

    return run, ok


WORKLOADS = {"sliding": _sliding, "batched": _batched}


def _time(torch, run, reps):
    run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(workload: str, rows: int = 1 << 24, reps: int = 5, passes: int = 2, log=print):
    import torch
    dev = torch.device("cuda:0")
    run, ok = WORKLOADS[workload](torch, dev, rows)
    best = dict(DEFAULT)
    lms.set_tuning(**best)
    best_ms = _time(torch, run, reps)
    if not ok():
        raise RuntimeError(f"{workload}: the default tuning reports a device status")
    base_ms = best_ms
    tried = {tuple(best.values()): best_ms}
    log(f"{workload}: default {best_ms:.4f} ms")
    for _ in range(passes):
        changed = False
        for coord in COORDS:
            for v in _values(coord):
                cand = dict(best, **dict(zip(coord, v)))
                key = tuple(cand.values())
                if key not in tried:
                    lms.set_tuning(**cand)
                    tried[key] = _time(torch, run, reps)
                    if not ok():
                        tried[key] = float("inf")
                    log(f"{workload}: {cand} {tried[key]:.4f} ms")
                if tried[key] < best_ms * 0.99:
                    best, best_ms, changed = cand, tried[key], True
        if not changed:
            break
    lms.set_tuning()
    return {"params": best, "ms": round(best_ms, 4), "default_ms": round(base_ms, 4), "evaluated": len(tried)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", nargs="+", default=list(WORKLOADS))
    ap.add_argument("--rows", type=int, default=1 << 24)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=PACKAGED)
    args = ap.parse_args()
    import torch
    out = {}
    if os.path.exists(args.out):
        with open(args.out) as f:
            out = json.load(f)

    def log(m):
        print(f"[autotune] {m}", file=sys.stderr, flush=True)

    for w in args.workload:
        t0 = time.perf_counter()
        r = tune(w, args.rows, args.reps, log=log)
        r["device"] = torch.cuda.get_device_name(0)
        r["seconds"] = round(time.perf_counter() - t0, 1)
        out[w] = r
        with open(args.out, "w") as f:
            json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

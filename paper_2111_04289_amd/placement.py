"""Learned CPU/GPU placement: timing records, training, evaluation.

MapDevice (Algorithm 2) decides per operation whether the CPU or the GPU runs
it; the paper's device costs are analytic (Eq. 7-9, with the inflection point
of Sec. III-D refit by the regression of Eq. 10).  Here a small MLP learns the
costs instead, from timings this engine records:

* ``collect`` runs an operation on sampled micro-batches on both devices and
  records (features, CPU ms, GPU ms).  GPU time includes copying the
  operation's input columns to HBM and its result back (stream data arrives
  in host memory), CPU time is the CPU execution function on ``cores``
  threads.  CPU runs above ``cpu_max_rows`` rows are skipped (masked in the
  loss).
* ``train`` fits log(ms) with the library's GPU training kernels (Adam).
* ``evaluate`` compares, on held-out batches, the measured runtime of the
  placements the learned model and the analytic model choose.

Run as ``python -m paper_2111_04289_amd.placement`` to collect, train and
evaluate on this machine; it prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import datagen, lms

MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "placement_mlp.npy")

OPS = ("fp", "tumble", "slide", "join")


def load_model(path: str | None = None):
    """The packaged trained parameters (float32), or None if there are none."""
    path = path or MODEL_PATH
    if not os.path.exists(path):
        return None
    p = np.load(path).astype(np.float32)
    return p if p.size == lms.MLP_NPARAMS else None
KIND = {"fp": lms.OP_FILTER, "tumble": lms.OP_AGG, "slide": lms.OP_AGG, "join": lms.OP_JOIN}
WINDOWS = ((10, 1), (30, 5), (30, 10), (60, 10), (60, 5))  # range/slide shapes of the paper's queries (s)
COLS_READ = {"fp": 3, "tumble": 4, "slide": 4, "join": 1}


class Pool:
    """Host (pinned) column pools from which micro-batches are sliced."""

    def __init__(self, rows: int, static_rows: int = 1 << 16, seed: int = 7):
        c = datagen.config1(rows, seed=seed)
        self.cols = [torch.from_numpy(x).pin_memory() for x in c]
        self.rows = rows
        bk, bp = datagen.static_table(static_rows)
        self.bk, self.bp = torch.from_numpy(bk), torch.from_numpy(bp)
        self.dtable = lms.lms_join_build(self.bk.cuda(), self.bp.cuda())
        self.dtable.max_mult()

    def batch(self, rng, n):
        off = int(rng.integers(0, self.rows - n + 1))
        return [c[off:off + n] for c in self.cols]


def sample_config(rng, max_rows):
    op = OPS[int(rng.integers(0, len(OPS)))]
    n = int(math.exp(rng.uniform(math.log(1024), math.log(max_rows))))
    sel = float(rng.choice([0.001, 0.05, 0.3, 0.6, 0.95]))
    w, s = WINDOWS[int(rng.integers(0, len(WINDOWS)))]
    if op == "tumble":
        w, s = (1, 0)
    if op in ("fp", "join"):
        w, s = (0, 0)
    return {"op": op, "rows": n, "sel": sel, "window_s": w, "slide_s": s}


def _query(cfg):
    cut = int(cfg["sel"] * (1 << 20))
    preds = [(2, lms.LT, cut)]
    if cfg["op"] == "tumble":
        return preds, [(2, 2, 0)], [(lms.COUNT, 0), (lms.SUM, 4)], lms.Window(0, 1000, 0, 0)
    aggs = [(lms.COUNT, 0), (lms.SUM, 2), (lms.MIN, 2), (lms.MAX, 2), (lms.AVG, 3)]
    return preds, [], aggs, lms.Window(0, int(cfg["window_s"] * 1000), int(cfg["slide_s"] * 1000), 0)


def run_gpu(pool, cfg, cols):
    """Wall time (ms) of the operation on the GPU, transfers included."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if cfg["op"] == "join":
        k = cols[1].cuda(non_blocking=True)
        i, p, d = lms.lms_hash_join(pool.dtable, k, cap=len(k) * max(1, pool.dtable.max_mult()))
        m = int(d[0])
        i[:m].cpu(), p[:m].cpu()
    elif cfg["op"] == "fp":
        dc = [c.cuda(non_blocking=True) for c in cols[:3]]
        preds, _, _, _ = _query(cfg)
        out, d = lms.lms_filter_project(dc, preds, [0, 1], [(2, 2, 0)])
        m = int(d[0])
        [o[:m].cpu() for o in out]
    else:
        dc = [c.cuda(non_blocking=True) for c in cols]
        preds, projs, aggs, w = _query(cfg)
        g, d = lms.lms_window_agg(dc, 1, w, aggs, preds, projs, cap=len(cols[0]) * max(1, w.length // (w.slide or w.length)))
        m = min(int(d[0]), g.cap)
        g.key[:m].cpu(), g.wstart[:m].cpu(), [a[:m].cpu() for a in g.aggs]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def run_cpu(pool, cfg, cols, cores):
    t0 = time.perf_counter()
    if cfg["op"] == "join":
        lms.lms_cpu_hash_join(pool.bk, pool.bp, cols[1], cap=len(cols[1]), nthreads=cores)
    elif cfg["op"] == "fp":
        preds, _, _, _ = _query(cfg)
        lms.lms_cpu_filter_project(cols[:3], preds, [0, 1], [(2, 2, 0)], nthreads=cores)
    else:
        preds, projs, aggs, w = _query(cfg)
        lms.lms_cpu_window_agg(cols, 1, w, aggs, preds, projs, nthreads=cores)
    return (time.perf_counter() - t0) * 1e3


def features(cfg, transfer=1, interval_s=0.0):
    n = cfg["rows"]
    distinct = min(int(n * cfg["sel"]) + 1, 1 << 20)
    return lms.mlp_features(KIND[cfg["op"]], n, COLS_READ[cfg["op"]], cfg["sel"], distinct, cfg["window_s"],
                            cfg["slide_s"], interval_s, transfer)


def collect(pool, n_records, seed, cores, cpu_max_rows, max_rows, log=None, cpu_every=1):
    """Timing records; the CPU side is timed on every cpu_every-th record (and
    only up to cpu_max_rows rows), the others keep it masked."""
    rng = np.random.default_rng(seed)
    recs = []
    t_start = time.perf_counter()
    for r in range(n_records):
        cfg = sample_config(rng, max_rows)
        cols = pool.batch(rng, cfg["rows"])
        g = run_gpu(pool, cfg, cols)
        c = run_cpu(pool, cfg, cols, cores) if cfg["rows"] <= cpu_max_rows and r % cpu_every == 0 else float("nan")
        recs.append(dict(cfg, gpu_ms=g, cpu_ms=c))
        if log and (r + 1) % 500 == 0:
            log(f"{r + 1} records in {time.perf_counter() - t_start:.1f} s")
    return recs


def to_arrays(recs):
    x = np.stack([features(r) for r in recs]).astype(np.float32)
    t = np.zeros((len(recs), 2), np.float32)
    m = np.zeros((len(recs), 2), np.float32)
    for i, r in enumerate(recs):
        for j, key in enumerate(("cpu_ms", "gpu_ms")):
            if np.isfinite(r[key]):
                t[i, j] = math.log(max(r[key], 1e-3))
                m[i, j] = 1.0
    return x, t, m


def train(recs, epochs=400, lr=3e-3, seed=0):
    x, t, m = to_arrays(recs)
    net = lms.Mlp(seed=seed)
    X, T, M = (torch.from_numpy(a).cuda() for a in (x, t, m))
    losses = []
    for e in range(epochs):
        net.loss_grad_async(X, T, M)
        net.adam(lr=lr)
        if e % 50 == 0 or e == epochs - 1:
            torch.cuda.synchronize()
            losses.append(float(net.loss.item()))
    return net, losses


def analytic_choice(cfg, cores):
    bytes_per_row = 4 * COLS_READ[cfg["op"]] + (4 if cfg["op"] != "join" else 4)
    devs, _ = lms.lms_plan([KIND[cfg["op"]]], cfg["rows"] * bytes_per_row, cores)
    return devs[0]


def learned_choice(cfg, params, cores):
    devs, _ = lms.lms_plan([KIND[cfg["op"]]], max(1, cfg["rows"] * 24), cores, mode=lms.PLAN_LEARNED, model=params,
                           rows=cfg["rows"], selectivity=cfg["sel"],
                           distinct_keys=min(int(cfg["rows"] * cfg["sel"]) + 1, 1 << 20),
                           ncols=[COLS_READ[cfg["op"]]], window_s=[cfg["window_s"]], slide_s=[cfg["slide_s"]])
    return devs[0]


def evaluate(recs, params, cores):
    """Measured total runtime of each policy's choices on records timed on both devices."""
    both = [r for r in recs if np.isfinite(r["cpu_ms"])]
    tot = {"learned": 0.0, "analytic": 0.0, "best": 0.0, "all_gpu": 0.0, "all_cpu": 0.0}
    wrong = {"learned": 0, "analytic": 0}
    for r in both:
        ms = {lms.DEV_CPU: r["cpu_ms"], lms.DEV_GPU: r["gpu_ms"]}
        best = lms.DEV_CPU if r["cpu_ms"] < r["gpu_ms"] else lms.DEV_GPU
        a = analytic_choice(r, cores)
        l = learned_choice(r, params, cores)
        tot["analytic"] += ms[a]
        tot["learned"] += ms[l]
        tot["best"] += ms[best]
        tot["all_gpu"] += r["gpu_ms"]
        tot["all_cpu"] += r["cpu_ms"]
        wrong["analytic"] += a != best
        wrong["learned"] += l != best
    return {"n": len(both), "total_ms": {k: round(v, 2) for k, v in tot.items()}, "mispredictions": wrong}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--records", type=int, default=6000)
    ap.add_argument("--heldout", type=int, default=600)
    ap.add_argument("--cores", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--pool-rows", type=int, default=1 << 24)
    ap.add_argument("--cpu-max-rows", type=int, default=1 << 22)
    ap.add_argument("--cpu-every", type=int, default=1, help="time the CPU side on every k-th training record only")
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--save", default=None, help="write the trained parameters (.npy) and records (.json) here")
    args = ap.parse_args()

    def log(msg):
        print(f"[placement] {msg}", file=sys.stderr, flush=True)

    log(f"pool of {args.pool_rows} rows, {args.cores} cores")
    pool = Pool(args.pool_rows)
    for cfg in ({"op": o, "rows": 4096, "sel": 0.3, "window_s": 10, "slide_s": 1} for o in OPS):  # warm up
        cols = pool.batch(np.random.default_rng(0), 4096)
        run_gpu(pool, cfg, cols)
        run_cpu(pool, cfg, cols, args.cores)
    recs = collect(pool, args.records, 1, args.cores, args.cpu_max_rows, args.pool_rows, log, args.cpu_every)
    held = collect(pool, args.heldout, 2, args.cores, args.cpu_max_rows, args.cpu_max_rows, log)
    log("training")
    t0 = time.perf_counter()
    net, losses = train(recs, epochs=args.epochs)
    train_s = time.perf_counter() - t0
    params = net.get_params()
    res = {"records": len(recs), "cpu_timed": int(sum(np.isfinite(r["cpu_ms"]) for r in recs)),
           "heldout": evaluate(held, params, args.cores), "train_seconds": round(train_s, 2),
           "loss": [round(v, 4) for v in losses], "cores": args.cores}
    if args.save:
        np.save(args.save + ".npy", params)
        json.dump(recs + held, open(args.save + ".records.json", "w"))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

"""Serving loop: continuous micro-batching of concurrent stream queries.

Datasets (1000-row files, Sec. V-A) arrive as a Poisson stream whose rate
steps through a schedule.  Each query owns an admission controller
(ConstructMicroBatch, Algorithm 1 with Eq. 6; ``lms.Admission``), a HIP stream
and a bounded number of in-flight micro-batches:

* every 10 ms the controller of each query with a free slot sees the datasets
  that arrived since its last poll and decides whether the buffered ones form
  the next micro-batch (dynamic micro-batch size under the query's latency
  bound);
* an admitted micro-batch starts once the HBM it needs (inputs, outputs,
  workspace) fits the budget left by the batches in flight (admission by free
  HBM); meanwhile later arrivals keep buffering;
* batches of different queries overlap on the device (one stream each); the
  two stateful window queries keep their partial aggregates on the device
  between micro-batches (``lms.WindowState``) and emit each window once the
  watermark (the newest dataset's creation time) passes its end;
* MapDevice (Algorithm 2; learned or analytic ``lms_plan``) places each batch
  of the stateless queries on the CPU (the library's CPU execution functions,
  in a worker thread, on the host-resident data) or on the GPU (copy in, HIP
  kernels, copy the result out).

A dataset's latency is the time from its creation to the moment its
micro-batch's result is back in host memory (end-to-end latency, Sec. V-B);
a batch's MaxLat is Eq. 5.  The plain per-batch form for comparison buffers
for a fixed trigger interval and then runs every query's batch on the GPU, one
launch chain after another on one stream (the paper's baseline with a
slide-sized trigger).

    python -m paper_2111_04289_amd.serve --step-s 30          # full rate schedule
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import datagen, lms

DS_ROWS = 1000
QUERIES = ("fp", "tumble", "slide", "join")
FP_CUT = datagen.CONFIG1_VAL_CUT  # val < 314573: selectivity 0.3
SLIDE_AGGS = [(lms.COUNT, 0), (lms.SUM, 2), (lms.MIN, 2), (lms.MAX, 2), (lms.AVG, 3)]
TUMBLE_AGGS = [(lms.COUNT, 0)]
IN_BYTES = {"fp": 20, "tumble": 16, "slide": 24, "join": 8}  # device input bytes per row
MAX_EMIT_WINDOWS = 8
# the operation chain of each query as the learned cost model sees it:
# (kind, columns read, window s, slide s), selectivity
SIZING_OPS = {"fp": ([(lms.OP_FILTER, 3, 0.0, 0.0)], 0.3), "tumble": ([(lms.OP_AGG, 4, 1.0, 0.0)], 1.0),
              "slide": ([(lms.OP_AGG, 4, 10.0, 1.0)], 0.3), "join": ([(lms.OP_JOIN, 1, 0.0, 0.0)], 1.0)}


# ---- traffic ------------------------------------------------------------------------

@dataclass
class Traffic:
    """Poisson dataset arrivals: for each step, a rate in rows/s held for step_s."""
    rates: tuple = (0.1e6, 1e6, 5e6, 10e6)
    step_s: float = 30.0
    ds_rows: int = DS_ROWS
    seed: int = 4

    def arrivals_ms(self) -> np.ndarray:
        rng = np.random.default_rng(self.seed)
        out, t0 = [], 0.0
        span = self.step_s * 1000.0
        for r in self.rates:
            n = int(rng.poisson(r / self.ds_rows * self.step_s))
            out.append(np.sort(rng.uniform(t0, t0 + span, n)))
            t0 += span
        return np.concatenate(out) if out else np.zeros(0)


class StreamData:
    """Host-resident (pinned) rows of the stream: dataset d holds stream rows
    [d * ds_rows, (d + 1) * ds_rows) whose ts is the dataset's creation time in
    ms; key, val and f are taken cyclically from a pool of config-1 rows."""

    def __init__(self, arrivals_ms: np.ndarray, pool_rows: int, ds_rows: int = DS_ROWS, seed: int = 1):
        cols = datagen.config1(pool_rows, seed=seed)
        pin = (lambda t: t.pin_memory()) if torch.cuda.is_available() else (lambda t: t)
        self.key = pin(torch.from_numpy(cols[1]))
        self.val = pin(torch.from_numpy(cols[2]))
        self.f = pin(torch.from_numpy(cols[3]))
        self.pool = pool_rows
        self.ds_rows = ds_rows
        self.arr = arrivals_ms
        self.ts_ds = np.floor(arrivals_ms).astype(np.int64)
        self.ts = pin(torch.from_numpy(np.repeat(self.ts_ds, ds_rows)))

    def segments(self, d0: int, d1: int):
        """(stream offset, pool lo, pool hi) pieces of the rows of datasets [d0, d1)."""
        lo, hi = d0 * self.ds_rows, d1 * self.ds_rows
        out, r = [], lo
        while r < hi:
            p = r % self.pool
            n = min(hi - r, self.pool - p)
            out.append((r - lo, p, p + n))
            r += n
        return out

    def host_cols(self, d0: int, d1: int, which=(0, 1, 2, 3)):
        """Contiguous host tensors of the columns `which` (0 ts, 1 key, 2 val, 3 f)."""
        lo, hi = d0 * self.ds_rows, d1 * self.ds_rows
        seg = self.segments(d0, d1)
        out = []
        for c in which:
            if c == 0:
                out.append(self.ts[lo:hi])
                continue
            src = (self.key, self.val, self.f)[c - 1]
            out.append(src[seg[0][1]:seg[0][2]] if len(seg) == 1 else torch.cat([src[a:b] for _, a, b in seg]))
        return out

    def dev_cols(self, d0: int, d1: int, which, device):
        """Device copies of the columns `which`, enqueued on the current stream."""
        lo, hi = d0 * self.ds_rows, d1 * self.ds_rows
        seg = self.segments(d0, d1)
        out = []
        for c in which:
            if c == 0:
                out.append(self.ts[lo:hi].to(device, non_blocking=True))
                continue
            src = (self.key, self.val, self.f)[c - 1]
            d = torch.empty(hi - lo, dtype=src.dtype, device=device)
            for off, a, b in seg:
                d[off:off + b - a].copy_(src[a:b], non_blocking=True)
            out.append(d)
        return out


# ---- per-query execution --------------------------------------------------------------

@dataclass
class Batch:
    q: str
    d0: int
    d1: int
    rows: int
    t_admit: float
    oldest: float
    need: int = 0
    device: int = lms.DEV_GPU
    stage: int = 0
    pred_proc: float = 0.0  # the controller's Eq. 6 processing term at admission (0: none yet)
    infpt: float = 0.0      # InfPT the analytic MapDevice ran with (Eq. 10 tuning)
    ev: object = None
    keep: list = field(default_factory=list)
    future: object = None
    result: object = None
    t_done: float = 0.0


class Query:
    def __init__(self, name, eng):
        self.name = name
        self.eng = eng
        # one stream per query (default priority); the plain form shares one
        self.stream = eng.shared_stream if eng.mode == "baseline" else torch.cuda.Stream()
        self.ws = lms.Workspace(eng.dev)
        self.next_ds = 0        # first dataset not yet offered to the controller
        self.next_batch_ds = 0  # first dataset not yet in an admitted batch
        self.waiting = []       # admitted batches waiting for HBM
        self.inflight = []
        self.lat = []           # per-dataset end-to-end latency (ms)
        self.maxlat = []        # per-batch MaxLat (ms)
        self.bound = []         # the latency bound each batch is held to (ms)
        self.est_err = []       # |predicted - measured| / measured processing time per batch
        self.proc = []
        self.batch_rows = []
        # time spent per step, as in the paper's overhead breakdown (ms):
        # datasets buffered before admission, host time in the admission
        # controller and in MapDevice
        self.t_buffer = 0.0
        self.t_construct = 0.0
        self.t_map = 0.0
        self.cpu_batches = 0
        self.rows_done = 0
        self.results = [] if eng.collect else None
        if eng.mode == "served":
            if name == "slide":
                self.ctl = lms.Admission(slide_ms=1000.0, poll_ms=eng.poll_ms)
            elif name == "tumble":
                self.ctl = lms.Admission(slide_ms=0.0, poll_ms=eng.poll_ms)
            else:
                self.ctl = lms.Admission(deadline_ms=eng.bound_ms, poll_ms=eng.poll_ms)
            if eng.sizing == "learned":
                # learned micro-batch sizing: Eq. 6's processing term from the cost model
                ops, sel = SIZING_OPS[name]
                self.ctl.set_model(eng.model, ops, selectivity=sel, distinct_keys=1 << 20, num_cores=eng.cores,
                                   bytes_per_row=IN_BYTES[name])
        # analytic MapDevice without a trained model: InfPT tuned online (Eq. 10)
        self.infpt = lms.InfPTTuner(seed=QUERIES.index(name)) if eng.model is None else None
        self.state = None
        self.drained = False
        self.closed = False  # the end-of-stream batch has taken the controller's buffer
        if name == "slide":
            self.state = lms.WindowState(lms.Window(0, 10000, 1000, 0), SLIDE_AGGS, eng.max_keys, 64, eng.dev,
                                         self.stream)
        elif name == "tumble":
            self.state = lms.WindowState(lms.Window(0, 1000, 0, 0), TUMBLE_AGGS, eng.max_keys, 16, eng.dev,
                                         self.stream)
        self.state_bytes = self.state.nbytes if self.state is not None else 0

    # bytes of HBM a batch of n rows holds while in flight
    def need(self, n):
        if self.name == "fp":
            return n * (IN_BYTES["fp"] + 20) + int(lms._lib.lms_filter_project_workspace(n))
        if self.name == "join":
            return n * (IN_BYTES["join"] + 8 * max(1, self.eng.join_mult)) + int(lms._lib.lms_hash_join_workspace(n))
        nagg = len(SLIDE_AGGS if self.name == "slide" else TUMBLE_AGGS)
        return n * IN_BYTES[self.name] + self.eng.max_keys * MAX_EMIT_WINDOWS * (16 + 8 * nagg)


class Engine:
    def __init__(self, data: StreamData, mode="served", queries=QUERIES, poll_ms=10.0, bound_ms=1000.0,
                 trigger_ms=1000.0, slots=2, hbm_budget=None, model=None, cores=None, max_keys=1 << 20,
                 collect=False, placement=True, sizing="learned", log=None):
        self.data, self.mode = data, mode
        self.sizing = sizing if model is not None else "analytic"
        self.poll_ms, self.bound_ms, self.trigger_ms = poll_ms, bound_ms, trigger_ms
        self.slots = slots
        self.model = model
        self.placement = placement and mode == "served"
        self.cores = cores or min(16, os.cpu_count() or 1)
        self.max_keys = max_keys
        self.collect = collect
        self.log = log or (lambda m: None)
        self.dev = torch.device("cuda")
        self.shared_stream = torch.cuda.Stream()
        bk, bp = datagen.static_table(1 << 20)
        self.bk, self.bp = torch.from_numpy(bk), torch.from_numpy(bp)
        self.table = lms.lms_join_build(self.bk.to(self.dev), self.bp.to(self.dev))
        self.join_mult = self.table.max_mult()
        self.queries = {q: Query(q, self) for q in queries}
        free, _ = torch.cuda.mem_get_info()
        state = sum(q.state_bytes for q in self.queries.values())
        self.budget = int(hbm_budget) if hbm_budget is not None else int(0.8 * free)
        self.reserved = 0
        self.hbm_waits = 0
        self.pool = ThreadPoolExecutor(max_workers=2)
        self.log(f"{mode}: HBM budget {self.budget / 2**30:.1f} GiB (window state {state / 2**30:.2f} GiB)")
        torch.cuda.synchronize()
        self.t0 = time.perf_counter()
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev0.record()
        torch.cuda.synchronize()
        self.t0_ev = (time.perf_counter() - self.t0) * 1e3  # host ms at which ev0 completed (upper bound)

    def now(self):
        return (time.perf_counter() - self.t0) * 1e3

    def batch_bound(self, q):
        """The latency bound a batch of q is held to: SlideTime for the sliding
        window, the window length for the tumbling one (its admission target, the
        mean past MaxLat of Eq. 3, moves with the batches themselves), and the
        deadline for the windowless queries."""
        if q.name in ("slide", "tumble"):
            return 1000.0
        return self.bound_ms

    def ev_ms(self, ev):
        return self.t0_ev + self.ev0.elapsed_time(ev)

    # ---- placement (MapDevice) ----------------------------------------------------------
    def place(self, q: Query, rows: int, interval_s: float, b=None):
        if not self.placement or q.name not in ("fp", "join"):
            return lms.DEV_GPU
        kind = lms.OP_FILTER if q.name == "fp" else lms.OP_JOIN
        ncols = 3 if q.name == "fp" else 1
        sel = 0.3 if q.name == "fp" else 1.0
        distinct = min(int(rows * sel) + 1, 1 << 20)
        if self.model is not None:
            devs, _ = lms.lms_plan([kind], rows * 24, self.cores, mode=lms.PLAN_LEARNED, model=self.model, rows=rows,
                                   selectivity=sel, distinct_keys=distinct, ncols=[ncols], window_s=[0],
                                   slide_s=[0], interval_s=interval_s)
        else:
            infpt = q.infpt.next(self.batch_bound(q))
            if b is not None:
                b.infpt = infpt
            devs, _ = lms.lms_plan([kind], rows * (4 * ncols + 4), self.cores, infpt_bytes=infpt)
        return devs[0]

    # ---- batch execution ------------------------------------------------------------------
    def start(self, q: Query, b: Batch):
        if b.device == lms.DEV_CPU:
            q.cpu_batches += 1
            b.future = self.pool.submit(self._cpu, q, b)
            b.stage = 9
            return
        with torch.cuda.stream(q.stream):
            s = q.stream
            if q.name == "fp":
                d = self.data.dev_cols(b.d0, b.d1, (0, 1, 2), self.dev)
                out, cnt = lms.lms_filter_project(d, [(2, lms.LT, FP_CUT)], [0, 1], [(2, 2, 0)], workspace=q.ws,
                                                  stream=s)
                b.keep = [d, out, cnt]
            elif q.name == "join":
                (k,) = self.data.dev_cols(b.d0, b.d1, (1,), self.dev)
                i, p, cnt = lms.lms_hash_join(self.table, k, workspace=q.ws, stream=s)
                out = [i, p]
                b.keep = [k, out, cnt]
            else:
                d = self.data.dev_cols(b.d0, b.d1, (0, 1) if q.name == "tumble" else (0, 1, 2, 3), self.dev)
                if b.rows:
                    if q.name == "slide":
                        q.state.update(d, 1, [(2, lms.LT, FP_CUT)], stream=s)
                    else:
                        q.state.update(d, 1, stream=s)
                aggs = SLIDE_AGGS if q.name == "slide" else TUMBLE_AGGS
                g = lms.Groups(self.max_keys * MAX_EMIT_WINDOWS, aggs, self.dev)
                wm = int(self.data.ts_ds[b.d1 - 1]) if b.rows else 0
                g, cnt = q.state.emit(wm, flush=b.rows == 0, max_windows=MAX_EMIT_WINDOWS, groups=g, stream=s)
                out = [g.key, g.wstart] + g.aggs
                b.keep = [d, out, cnt, g]
            b.cnt_h = torch.empty(2, dtype=torch.int64, pin_memory=True)
            b.cnt_h.copy_(cnt, non_blocking=True)
            b.ev = torch.cuda.Event()
            b.ev.record(s)
            b.out_dev = out
            b.stage = 1

    def _cpu(self, q: Query, b: Batch):
        nt = max(1, self.cores // 2)
        if q.name == "fp":
            cols = self.data.host_cols(b.d0, b.d1, (0, 1, 2))
            out = lms.lms_cpu_filter_project(cols, [(2, lms.LT, FP_CUT)], [0, 1], [(2, 2, 0)], nthreads=nt)
        else:
            (k,) = self.data.host_cols(b.d0, b.d1, (1,))
            i, p, _ = lms.lms_cpu_hash_join(self.bk, self.bp, k, cap=len(k) * max(1, self.join_mult), nthreads=nt)
            out = [i, p]
        return out, self.now()

    def progress(self, q: Query, b: Batch) -> bool:
        """Advances b; returns True once its result is in host memory."""
        if b.stage == 9:
            if not b.future.done():
                return False
            b.result, b.t_done = b.future.result()
            return True
        if b.stage == 1:
            if not b.ev.query():
                return False
            m, status = int(b.cnt_h[0]), int(b.cnt_h[1])
            if status != 0:
                raise RuntimeError(f"{q.name}: device status {status}")
            with torch.cuda.stream(q.stream):
                b.result = []
                for t in b.out_dev:
                    h = torch.empty(m, dtype=t.dtype, pin_memory=True)
                    h.copy_(t[:m], non_blocking=True)
                    b.result.append(h)
                b.ev = torch.cuda.Event(enable_timing=True)
                b.ev.record(q.stream)
            b.stage = 2
            return False
        if b.stage == 2:
            if not b.ev.query():
                return False
            b.t_done = self.ev_ms(b.ev)
            b.keep = []
            b.out_dev = None
            return True
        return False

    def finish(self, q: Query, b: Batch):
        self.reserved -= b.need
        if b.rows == 0 and q.state is not None:  # a flush: drained once it emitted no window
            inf = q.state.info(stream=q.stream)
            q.drained = inf["emit_hi"] < inf["emit_lo"]
        arr = self.data.arr[b.d0:b.d1]
        if b.rows:
            lat = b.t_done - arr
            q.lat.append(lat)
            maxlat = float(lat.max())
            q.bound.append(self.batch_bound(q))
            if b.pred_proc > 0:
                q.est_err.append(abs(b.pred_proc - (b.t_done - b.t_admit)) / max(b.t_done - b.t_admit, 1e-3))
            q.maxlat.append(maxlat)
            q.proc.append(b.t_done - b.t_admit)
            q.t_buffer += max(0.0, b.t_admit - b.oldest)
            q.batch_rows.append(b.rows)
            q.rows_done += b.rows
            if self.mode == "served":
                q.ctl.done(b.rows, max(b.t_done - b.t_admit, 1e-3), maxlat)
                if q.infpt is not None and b.infpt > 0:  # Eq. 10's record of this batch
                    q.infpt.record(b.infpt, b.rows / max(b.t_done - b.t_admit, 1e-3), maxlat)
        if q.results is not None:
            q.results.append((b.d0, b.d1, [t.numpy() if hasattr(t, "numpy") else t for t in b.result]))

    # ---- main loop --------------------------------------------------------------------
    def run(self, drain_s=30.0, report_every_ms=10000.0):
        arr = self.data.arr
        nds = len(arr)
        end_ms = float(arr[-1]) if nds else 0.0
        next_report = report_every_ms
        next_poll = 0.0
        next_trigger = self.trigger_ms
        last_admit = {q: 0.0 for q in self.queries}
        while True:
            now = self.now()
            arrived = int(np.searchsorted(arr, now, side="right"))
            if now >= next_report:
                next_report += report_every_ms
                done = {q.name: (len(q.batch_rows), q.rows_done) for q in self.queries.values()}
                self.log(f"{self.mode} t={now / 1e3:.0f} s: {arrived} datasets arrived; (batches, rows) done {done}")
            # completions
            for q in self.queries.values():
                for b in list(q.inflight):
                    if self.progress(q, b):
                        q.inflight.remove(b)
                        self.finish(q, b)
            # admission
            if self.mode == "served" and now >= next_poll:
                next_poll = now + self.poll_ms
                for q in self.queries.values():
                    if q.closed or len(q.inflight) + len(q.waiting) >= self.slots:
                        continue
                    new = arr[q.next_ds:arrived]
                    t0 = time.perf_counter()
                    d = q.ctl.poll(now, new, np.full(len(new), DS_ROWS, np.int64))
                    q.t_construct += (time.perf_counter() - t0) * 1e3
                    q.next_ds = arrived
                    if d.admit:
                        d0 = q.next_batch_ds
                        d1 = d0 + int(d.datasets)
                        q.next_batch_ds = d1
                        b = Batch(q.name, d0, d1, (d1 - d0) * DS_ROWS, now, float(arr[d0]))
                        b.need = q.need(b.rows)
                        b.pred_proc = q.ctl.predict_ms(b.rows)
                        t0 = time.perf_counter()
                        b.device = self.place(q, b.rows, (now - last_admit[q.name]) / 1e3, b)
                        q.t_map += (time.perf_counter() - t0) * 1e3
                        last_admit[q.name] = now
                        q.waiting.append(b)
            elif self.mode == "baseline" and now >= next_trigger and not any(
                    q.inflight for q in self.queries.values()):
                next_trigger = max(next_trigger + self.trigger_ms, now)
                for q in self.queries.values():
                    d0, d1 = q.next_batch_ds, arrived
                    if d1 > d0:
                        q.next_batch_ds = d1
                        b = Batch(q.name, d0, d1, (d1 - d0) * DS_ROWS, now, float(arr[d0]))
                        b.need = q.need(b.rows)
                        q.waiting.append(b)
            # start admitted batches whose memory fits
            for q in self.queries.values():
                while q.waiting and len(q.inflight) < self.slots:
                    b = q.waiting[0]
                    if self.reserved + b.need > self.budget:
                        if self.reserved == 0:
                            raise RuntimeError(f"{q.name}: a batch of {b.rows} rows exceeds the HBM budget")
                        self.hbm_waits += 1
                        break
                    q.waiting.pop(0)
                    self.reserved += b.need
                    self.start(q, b)
                    q.inflight.append(b)
            # end of stream: flush window states once everything else is done
            all_in = arrived >= nds and now > end_ms
            if all_in:
                busy = False
                for q in self.queries.values():
                    if q.next_batch_ds < nds:
                        busy = True
                        if self.mode == "served" and not q.inflight and not q.waiting:
                            # deliver the rest regardless of the deadline; the
                            # controller's buffer is handed over with it
                            d0, d1 = q.next_batch_ds, nds
                            q.next_batch_ds = d1
                            q.next_ds = nds
                            q.closed = True
                            b = Batch(q.name, d0, d1, (d1 - d0) * DS_ROWS, now, float(arr[d0]))
                            b.need = q.need(b.rows)
                            q.waiting.append(b)
                    elif q.inflight or q.waiting:
                        busy = True
                    elif q.state is not None and not q.drained:
                        b = Batch(q.name, nds, nds, 0, now, now)  # flush: emits the windows still open
                        b.need = q.need(0)
                        q.waiting.append(b)
                        busy = True
                if not busy:
                    break
                if now > end_ms + drain_s * 1e3:
                    raise RuntimeError("serving loop did not drain")
            time.sleep(0.0005 if any(q.inflight for q in self.queries.values()) else 0.001)
        self.pool.shutdown()
        return self.report(end_ms)

    def report(self, end_ms):
        def breakdown(q):
            # shares of the query's time (the paper's overhead breakdown):
            # buffering before admission, the admission controller, MapDevice,
            # processing (admission to result on the host), and blocking on an
            # asynchronous optimizer -- zero here: the placement model is
            # evaluated synchronously, in microseconds
            parts = {"buffering": q.t_buffer, "construct_micro_batch": q.t_construct, "map_device": q.t_map,
                     "processing": float(np.sum(q.proc)) if q.proc else 0.0, "optimization_blocking": 0.0}
            tot = sum(parts.values()) or 1.0
            return {k: round(100.0 * v / tot, 3) for k, v in parts.items()}

        out = {"mode": self.mode, "sizing": self.sizing if self.mode == "served" else "fixed trigger",
               "stream_ms": round(end_ms, 1), "queries": {}}
        total = 0
        wall = self.now()
        for q in self.queries.values():
            lat = np.concatenate(q.lat) if q.lat else np.zeros(1)
            ml = np.array(q.maxlat) if q.maxlat else np.zeros(1)
            total += q.rows_done
            out["queries"][q.name] = {
                "batches": len(q.batch_rows), "rows": q.rows_done, "cpu_batches": q.cpu_batches,
                "mean_batch_rows": round(float(np.mean(q.batch_rows)), 1) if q.batch_rows else 0,
                "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
                "maxlat_p50_ms": round(float(np.percentile(ml, 50)), 2),
                "maxlat_p99_ms": round(float(np.percentile(ml, 99)), 2),
                "mean_proc_ms": round(float(np.mean(q.proc)), 3) if q.proc else 0.0,
                # batches whose MaxLat (Eq. 5) exceeded the bound they were admitted under
                "over_bound_pct": round(100.0 * float(np.mean(np.array(q.maxlat) > np.array(q.bound))), 2)
                if q.maxlat else 0.0,
                # median relative error of the admission's processing-time estimate
                "proc_est_err_pct": round(100.0 * float(np.median(q.est_err)), 1) if q.est_err else None,
                "breakdown_pct": breakdown(q)}
        out["rows_per_query"] = total // max(1, len(self.queries))
        out["Mrows_s"] = round(total / max(1, len(self.queries)) / (wall / 1e3) / 1e6, 3)
        out["wall_s"] = round(wall / 1e3, 2)
        all_lat = np.concatenate([np.concatenate(q.lat) for q in self.queries.values() if q.lat])
        out["p50_ms"] = round(float(np.percentile(all_lat, 50)), 2)
        out["p99_ms"] = round(float(np.percentile(all_lat, 99)), 2)
        out["hbm_waits"] = self.hbm_waits
        return out


def serve(traffic: Traffic, mode="served", pool_rows=1 << 24, queries=QUERIES, model=None, log=None, **kw):
    arr = traffic.arrivals_ms()
    data = StreamData(arr, pool_rows, traffic.ds_rows)
    eng = Engine(data, mode=mode, queries=queries, model=model, log=log, **kw)
    res = eng.run()
    return res, eng


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", type=float, nargs="+", default=[0.1e6, 1e6, 5e6, 10e6])
    ap.add_argument("--step-s", type=float, default=30.0)
    ap.add_argument("--pool-rows", type=int, default=1 << 24)
    ap.add_argument("--mode", nargs="+", default=["served", "baseline"])
    ap.add_argument("--model", default=None, help="MLP parameters (.npy) for learned placement")
    ap.add_argument("--no-placement", action="store_true")
    ap.add_argument("--bound-ms", type=float, default=1000.0, help="latency bound of the windowless queries")
    ap.add_argument("--sizing", default="learned", choices=("learned", "analytic"),
                    help="Eq. 6 processing term: the learned cost model, or Eq. 4's AvgThPut")
    args = ap.parse_args()

    def log(m):
        print(f"[serve] {m}", file=sys.stderr, flush=True)

    model = np.load(args.model).astype(np.float32) if args.model else None
    out = {}
    for mode in args.mode:
        t = Traffic(tuple(args.rates), args.step_s)
        log(f"{mode}: rates {args.rates} rows/s, {args.step_s} s each")
        res, _ = serve(t, mode, args.pool_rows, model=model, log=log, placement=not args.no_placement,
                       sizing=args.sizing, bound_ms=args.bound_ms)
        log(json.dumps(res))
        out[mode] = res
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

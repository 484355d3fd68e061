"""CPU oracle of the micro-batch operators -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and the
two share no code: this package computes each result from its plain
definition (see ``lms_oracle.c``), the GPU library from panes, partitions and
LDS hash tables.

Functions take NumPy arrays in host memory and return NumPy arrays:

* :func:`filter_project`  -- Table II Filtering + Projection.
* :func:`window_agg`      -- Table II Aggregation (Hash) over the windows of
  Table I (SlideTime, 0 = tumbling) / Table III (range, slide); every row is
  assigned to each window it falls in (the Expand semantics), no panes.
* :func:`window_group`    -- the same definition evaluated for one output group.
* :func:`hash_join`       -- Table II Join (Hash), stream-static inner equi-join.
* :func:`window_query`    -- Table III's query shapes: a composite group key
  (LR2S), HAVING on an aggregate (LR2S), ORDER BY an aggregate (CM1).
* :func:`window_self_join` -- Table III's LR1: the stream joined with the rows
  of its own window on equal keys.
* :mod:`oracle.plan`      -- MapDevice (Algorithm 2) with Eq. 7-9.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lms_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

I32, I64, F32, F64 = 0, 1, 2, 3
LT, LE, GT, GE, EQ, NE = 0, 1, 2, 3, 4, 5
COUNT, SUM, MIN, MAX, AVG = 0, 1, 2, 3, 4

_DT = {np.dtype(np.int32): I32, np.dtype(np.int64): I64, np.dtype(np.float32): F32, np.dtype(np.float64): F64}


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _lib.orc_filter_project.restype = ctypes.c_int64
        _lib.orc_window_agg.restype = ctypes.c_int64
        _lib.orc_window_group.restype = ctypes.c_int64
        _lib.orc_hash_join.restype = ctypes.c_int64
        _lib.orc_window_agg_keys.restype = ctypes.c_int64
        _lib.orc_window_self_join.restype = ctypes.c_int64
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _i32s(xs):
    a = np.asarray(list(xs), dtype=np.int32)
    return a if a.size else np.zeros(1, np.int32)


def _i64s(xs):
    a = np.asarray(list(xs), dtype=np.int64)
    return a if a.size else np.zeros(1, np.int64)


def _f64s(xs):
    a = np.asarray(list(xs), dtype=np.float64)
    return a if a.size else np.zeros(1, np.float64)


class _Query:
    """Marshals columns, predicates and projections for the C oracle."""

    def __init__(self, cols, preds=(), projs=()):
        self.cols = [np.ascontiguousarray(c) for c in cols]
        n = {len(c) for c in self.cols}
        if len(n) > 1:
            raise ValueError("columns differ in length")
        self.n = n.pop() if n else 0
        self.dts = _i32s(_DT[c.dtype] for c in self.cols)
        self.colptrs = (ctypes.c_void_p * max(1, len(self.cols)))(*[c.ctypes.data for c in self.cols])
        preds = list(preds)
        self.npred = len(preds)
        self.pcol = _i32s(p[0] for p in preds)
        self.pop = _i32s(p[1] for p in preds)
        self.pival = _i64s(int(p[2]) for p in preds)
        self.pfval = _f64s(float(p[3]) if len(p) > 3 else float(p[2]) for p in preds)
        projs = list(projs)
        self.nproj = len(projs)
        self.prsrc = _i32s(p[0] for p in projs)
        self.prmul = _i64s(p[1] for p in projs)
        self.pradd = _i64s(p[2] for p in projs)

    def args(self):
        return [
            ctypes.c_int64(self.n), ctypes.c_int(len(self.cols)), self.colptrs, _ptr(self.dts),
            ctypes.c_int(self.npred), _ptr(self.pcol), _ptr(self.pop), _ptr(self.pival), _ptr(self.pfval),
        ]

    def proj_args(self):
        return [ctypes.c_int(self.nproj), _ptr(self.prsrc), _ptr(self.prmul), _ptr(self.pradd)]


def filter_project(cols, preds=(), keep=(), projs=()):
    """Rows passing every predicate, in input order: keep columns then projections.

    preds: (col, op, ival[, fval]); projs: (src, mul, add).  Integer outputs are
    returned with the source column's dtype, float outputs likewise.
    """
    lib = _load()
    q = _Query(cols, preds, projs)
    keep = list(keep)
    outs = []
    for c in keep:
        outs.append(np.zeros(q.n, np.int64 if q.cols[c].dtype.kind == "i" else np.float64))
    for p in projs:
        outs.append(np.zeros(q.n, np.int64))
    optrs = (ctypes.c_void_p * max(1, len(outs)))(*[o.ctypes.data for o in outs])
    kp = _i32s(keep)
    m = lib.orc_filter_project(*q.args(), ctypes.c_int(len(keep)), _ptr(kp), *q.proj_args(), optrs)
    res = []
    for j, o in enumerate(outs):
        src = q.cols[keep[j]] if j < len(keep) else q.cols[projs[j - len(keep)][0]]
        res.append(o[:m].astype(src.dtype))
    return res


def window_agg(cols, key_col, ts_col, length, slide=0, origin=0, aggs=((COUNT, 0),), preds=(), projs=()):
    """All (key, window) groups sorted by (window start, key).

    Returns dict(key=int64[G], wstart=int64[G], aggs=[int64 or float64 arrays]).
    """
    lib = _load()
    q = _Query(cols, preds, projs)
    aggs = list(aggs)
    afn = _i32s(a[0] for a in aggs)
    acol = _i32s(a[1] for a in aggs)
    cap = 1024
    while True:
        ok = np.zeros(cap, np.int64)
        ow = np.zeros(cap, np.int64)
        oi = np.zeros(max(1, len(aggs)) * cap, np.int64)
        of = np.zeros(max(1, len(aggs)) * cap, np.float64)
        g = lib.orc_window_agg(*q.args(), *q.proj_args(), ctypes.c_int(key_col), ctypes.c_int(ts_col),
                               ctypes.c_int64(length), ctypes.c_int64(slide), ctypes.c_int64(origin),
                               ctypes.c_int(len(aggs)), _ptr(afn), _ptr(acol), ctypes.c_int64(cap), _ptr(ok),
                               _ptr(ow), _ptr(oi), _ptr(of))
        if g < 0:
            raise MemoryError("oracle window_agg ran out of memory")
        if g <= cap:
            break
        cap = int(g)
    out = []
    for k, (fn, _) in enumerate(aggs):
        out.append(of[k * cap:k * cap + g].copy() if fn == AVG else oi[k * cap:k * cap + g].copy())
    return {"key": ok[:g].copy(), "wstart": ow[:g].copy(), "aggs": out}


def window_group(cols, key_col, ts_col, length, slide, origin, aggs, qkey, qws, preds=(), projs=()):
    """Aggregates of the single group (qkey, window starting at qws)."""
    lib = _load()
    q = _Query(cols, preds, projs)
    aggs = list(aggs)
    afn = _i32s(a[0] for a in aggs)
    acol = _i32s(a[1] for a in aggs)
    oi = np.zeros(max(1, len(aggs)), np.int64)
    of = np.zeros(max(1, len(aggs)), np.float64)
    cnt = lib.orc_window_group(*q.args(), *q.proj_args(), ctypes.c_int(key_col), ctypes.c_int(ts_col),
                               ctypes.c_int64(length), ctypes.c_int64(slide), ctypes.c_int64(origin),
                               ctypes.c_int(len(aggs)), _ptr(afn), _ptr(acol), ctypes.c_int64(qkey),
                               ctypes.c_int64(qws), _ptr(oi), _ptr(of))
    vals = [of[k] if fn == AVG else oi[k] for k, (fn, _) in enumerate(aggs)]
    return int(cnt), vals


def hash_join(build_keys, build_payload, probe_keys):
    """Inner equi-join pairs (probe index int64, payload int32) in (i, j) order."""
    lib = _load()
    bk = np.ascontiguousarray(build_keys)
    bp = np.ascontiguousarray(build_payload, dtype=np.int32)
    pk = np.ascontiguousarray(probe_keys)
    cap = max(1024, len(pk))
    while True:
        oi = np.zeros(cap, np.int64)
        op = np.zeros(cap, np.int32)
        m = lib.orc_hash_join(ctypes.c_int64(len(bk)), _ptr(bk), ctypes.c_int(_DT[bk.dtype]), _ptr(bp),
                              ctypes.c_int64(len(pk)), _ptr(pk), ctypes.c_int(_DT[pk.dtype]), ctypes.c_int64(cap),
                              _ptr(oi), _ptr(op))
        if m < 0:
            raise MemoryError("oracle hash_join ran out of memory")
        if m <= cap:
            return oi[:m].copy(), op[:m].copy()
        cap = int(m)


def _cmp(v, op, c):
    return {LT: v < c, LE: v <= c, GT: v > c, GE: v >= c, EQ: v == c, NE: v != c}[op]


def window_query(cols, key_cols, ts_col, length, slide=0, origin=0, aggs=((COUNT, 0),), preds=(), projs=(),
                 having=None, order_by=None):
    """Windowed group-by over the tuple of key columns ``key_cols`` (Table III
    LR2S: GROUPBY (highway, direction, segment)), then

    * ``having=(k, op, value)``: keep the groups whose aggregate k satisfies
      ``aggs[k] op value`` (LR2S: HAVING avgSpeed < 40.0);
    * ``order_by=(k, descending)``: rows of each window ordered by aggregate k
      (ascending unless descending), ties by the key tuple (CM1: ORDERBY
      SUM(cpu)); without it, rows are sorted by (window start, key tuple).

    Returns dict(keys=[int64[G] per key column], wstart=int64[G], aggs=[...]).
    """
    lib = _load()
    q = _Query(cols, preds, projs)
    aggs = list(aggs)
    key_cols = list(key_cols)
    nk = len(key_cols)
    kc = _i32s(key_cols)
    afn = _i32s(a[0] for a in aggs)
    acol = _i32s(a[1] for a in aggs)
    cap = 1024
    while True:
        ok = np.zeros(max(1, nk) * cap, np.int64)
        ow = np.zeros(cap, np.int64)
        oi = np.zeros(max(1, len(aggs)) * cap, np.int64)
        of = np.zeros(max(1, len(aggs)) * cap, np.float64)
        g = lib.orc_window_agg_keys(*q.args(), *q.proj_args(), ctypes.c_int(nk), _ptr(kc), ctypes.c_int(ts_col),
                                    ctypes.c_int64(length), ctypes.c_int64(slide), ctypes.c_int64(origin),
                                    ctypes.c_int(len(aggs)), _ptr(afn), _ptr(acol), ctypes.c_int64(cap), _ptr(ok),
                                    _ptr(ow), _ptr(oi), _ptr(of))
        if g == -2:
            raise ValueError("1 to 4 key columns")
        if g < 0:
            raise MemoryError("oracle window_query ran out of memory")
        if g <= cap:
            break
        cap = int(g)
    res = {"keys": [ok[j * cap:j * cap + g].copy() for j in range(nk)], "wstart": ow[:g].copy(),
           "aggs": [of[k * cap:k * cap + g].copy() if fn == AVG else oi[k * cap:k * cap + g].copy()
                    for k, (fn, _) in enumerate(aggs)]}
    if having is not None:
        k, op, value = having
        keep = _cmp(res["aggs"][k], op, value)
        res = {"keys": [a[keep] for a in res["keys"]], "wstart": res["wstart"][keep],
               "aggs": [a[keep] for a in res["aggs"]]}
    if order_by is not None:
        k, desc = order_by
        v = res["aggs"][k]
        # a stable sort: window start first, then the aggregate, then the key tuple
        order = np.lexsort(tuple(reversed(res["keys"])) + ((-v if desc else v), res["wstart"]))
        res = {"keys": [a[order] for a in res["keys"]], "wstart": res["wstart"][order],
               "aggs": [a[order] for a in res["aggs"]]}
    return res


def window_self_join(cols, key_col, ts_col, length, slide=0, origin=0, preds=()):
    """Every (window start, l, a) with rows l and a both passing, both in the
    window and of equal key (Table III LR1: A.vehicle == L.vehicle over A's
    range/slide window), in (window start, l, a) order."""
    lib = _load()
    q = _Query(cols, preds, ())
    cap = max(1024, q.n)
    while True:
        ow = np.zeros(cap, np.int64)
        ol = np.zeros(cap, np.int64)
        oa = np.zeros(cap, np.int64)
        m = lib.orc_window_self_join(*q.args(), ctypes.c_int(key_col), ctypes.c_int(ts_col),
                                     ctypes.c_int64(length), ctypes.c_int64(slide), ctypes.c_int64(origin),
                                     ctypes.c_int64(cap), _ptr(ow), _ptr(ol), _ptr(oa))
        if m < 0:
            raise MemoryError("oracle window_self_join ran out of memory")
        if m <= cap:
            return ow[:m].copy(), ol[:m].copy(), oa[:m].copy()
        cap = int(m)

"""Helpers for the GPU parity tests: run an operator through the C-ABI binding
and compare its result with the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np
import torch

import oracle

AVG_RTOL = 1e-5  # relative tolerance on AVG stated for the windowed aggregates


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(cols):
    return [torch.from_numpy(np.ascontiguousarray(c)).cuda() for c in cols]


def gpu_window_agg(cols_np, key_col, ts_col, length, slide, origin, aggs, preds=(), projs=(), cap=None, dev_cols=None):
    from paper_2111_04289_amd import lms
    dc = dev_cols if dev_cols is not None else to_dev(cols_np)
    g, d = lms.lms_window_agg(dc, key_col, lms.Window(ts_col, length, slide, origin), aggs, preds, projs, cap=cap)
    torch.cuda.synchronize()
    cnt, status = [int(x) for x in d.cpu()]
    m = min(cnt, g.cap)
    res = {"key": g.key[:m].cpu().numpy(), "wstart": g.wstart[:m].cpu().numpy(),
           "aggs": [a[:m].cpu().numpy() for a in g.aggs]}
    return res, cnt, status


def canonical(res):
    order = np.lexsort((res["key"], res["wstart"]))
    return {"key": res["key"][order], "wstart": res["wstart"][order], "aggs": [a[order] for a in res["aggs"]]}


def assert_window_equal(got, exp, aggs, what=""):
    g = canonical(got)
    e = canonical(exp)
    assert len(g["key"]) == len(e["key"]), f"{what}: {len(g['key'])} groups vs oracle {len(e['key'])}"
    np.testing.assert_array_equal(g["wstart"], e["wstart"], err_msg=what)
    np.testing.assert_array_equal(g["key"], e["key"], err_msg=what)
    for k, (fn, _) in enumerate(aggs):
        if fn == oracle.AVG:
            bad = ~(np.abs(g["aggs"][k] - e["aggs"][k]) <= AVG_RTOL * np.abs(e["aggs"][k]))
            assert not bad.any(), f"{what}: AVG differs in {int(bad.sum())} groups, e.g. {np.flatnonzero(bad)[:5]}"
        else:
            np.testing.assert_array_equal(g["aggs"][k], e["aggs"][k], err_msg=f"{what} agg {k}")

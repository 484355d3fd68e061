"""GPU parity of Table III's query shapes against the oracle: composite group
keys with HAVING (LR2S), ORDER BY an aggregate within each window (CM1), the
equality filter (CM2S), and the windowed self-join (LR1)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import AVG_RTOL, log, to_dev
from oracle import AVG, COUNT, EQ, GE, LE, LT, MAX, MIN, SUM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def lr_cols(seed, n, ts_hi=60000, nseg=100):
    """Linear Road-shaped rows: ts, highway 0..9, direction 0..1, segment,
    speed (quarter units, exact in double sums), vehicle id."""
    rng = np.random.default_rng(seed)
    ts = rng.integers(0, ts_hi, n, dtype=np.int64)
    hw = rng.integers(0, 10, n, dtype=np.int32)
    dr = rng.integers(0, 2, n, dtype=np.int64)
    seg = rng.integers(0, nseg, n, dtype=np.int32)
    speed = (rng.integers(0, 400, n) / 4.0).astype(np.float32)
    veh = rng.integers(0, 3000, n, dtype=np.int64)
    return [ts, hw, dr, seg, speed, veh]


KEYS = [(1, 0, 9), (2, 0, 1), (3, 0, 99)]


def gpu_query(lms, cols, keys, window, aggs, **kw):
    g, d = lms.lms_window_query(to_dev(cols), keys, window, aggs, **kw)
    torch.cuda.synchronize()
    cnt, status = [int(x) for x in d.cpu()]
    m = min(cnt, g.cap)
    return {"keys": [k[:m].cpu().numpy() for k in g.keys], "wstart": g.wstart[:m].cpu().numpy(),
            "aggs": [a[:m].cpu().numpy() for a in g.aggs]}, cnt, status


def canonical(res):
    order = np.lexsort(tuple(reversed(res["keys"])) + (res["wstart"],))
    return {"keys": [k[order] for k in res["keys"]], "wstart": res["wstart"][order],
            "aggs": [a[order] for a in res["aggs"]]}


def assert_query_equal(got, exp, aggs, ordered, what):
    if not ordered:
        got = canonical(got)
    assert len(got["wstart"]) == len(exp["wstart"]), what
    np.testing.assert_array_equal(got["wstart"], exp["wstart"], err_msg=what)
    for j, k in enumerate(exp["keys"]):
        np.testing.assert_array_equal(got["keys"][j], k, err_msg=f"{what} key {j}")
    for k, (fn, _) in enumerate(aggs):
        if fn == AVG:
            np.testing.assert_allclose(got["aggs"][k], exp["aggs"][k], rtol=AVG_RTOL, err_msg=f"{what} agg {k}")
        else:
            np.testing.assert_array_equal(got["aggs"][k], exp["aggs"][k], err_msg=f"{what} agg {k}")


@pytest.mark.parametrize("length,slide,having", [
    (30000, 5000, (1, LT, 40.0)),   # LR2S: AVG(speed) per (highway, direction, segment), HAVING avg < 40
    (30000, 10000, (1, LE, 40.0)),  # the boundary value itself kept (quarter speeds: exact averages)
    (1000, 0, (0, GE, 3)),          # tumbling, HAVING on COUNT
    (60000, 10000, None),
])
def test_composite_key_having(lms, length, slide, having):
    cols = lr_cols(1, 200_000)
    aggs = [(COUNT, 0), (AVG, 4), (MIN, 3), (MAX, 1)]
    w = lms.Window(0, length, slide, 0)
    log(f"composite key query len={length} slide={slide} having={having}")
    got, cnt, status = gpu_query(lms, cols, KEYS, w, aggs, having=having)
    assert status == 0
    exp = oracle.window_query(cols, [1, 2, 3], 0, length, slide, 0, aggs, having=having)
    assert cnt == len(exp["wstart"])
    assert_query_equal(got, exp, aggs, False, "composite")


def test_composite_key_with_predicate_projection_and_wide_values(lms):
    rng = np.random.default_rng(5)
    n = 120_000
    ts = rng.integers(-20000, 40000, n, dtype=np.int64)
    k0 = rng.integers(-(1 << 40), -(1 << 40) + 50, n, dtype=np.int64)  # a narrow domain far from zero
    k1 = rng.integers(7, 12, n, dtype=np.int32)
    val = rng.integers(0, 1 << 20, n, dtype=np.int32)
    cols = [ts, k0, k1, val]
    keys = [(1, -(1 << 40), -(1 << 40) + 49), (2, 7, 11)]
    aggs = [(SUM, 4), (COUNT, 0), (MAX, 3)]
    preds, projs = [(3, LT, 700_000)], [(3, 3, -5)]
    got, cnt, status = gpu_query(lms, cols, keys, lms.Window(0, 7000, 3000, 250), aggs, preds=preds, projs=projs,
                                 having=(0, GE, 1 << 22))
    assert status == 0
    exp = oracle.window_query(cols, [1, 2], 0, 7000, 3000, 250, aggs, preds=preds, projs=projs,
                              having=(0, GE, 1 << 22))
    assert cnt == len(exp["wstart"]) > 0
    assert_query_equal(got, exp, aggs, False, "wide composite")


@pytest.mark.parametrize("agg_k,desc", [(0, True), (1, False), (2, True)])
def test_order_by_aggregate(lms, agg_k, desc):
    """CM1: ORDER BY an aggregate within each window; ties keep key order."""
    cols = lr_cols(2, 150_000, nseg=40)
    aggs = [(SUM, 3), (AVG, 4), (COUNT, 0)]
    w = lms.Window(0, 20000, 10000, 0)
    log(f"order by agg {agg_k} desc={desc}")
    got, cnt, status = gpu_query(lms, cols, KEYS, w, aggs, order=(agg_k, desc))
    assert status == 0
    exp = oracle.window_query(cols, [1, 2, 3], 0, 20000, 10000, 0, aggs, order_by=(agg_k, desc))
    assert cnt == len(exp["wstart"])
    assert_query_equal(got, exp, aggs, True, "ordered")


def test_order_by_single_key_with_having(lms):
    """CM1-shaped: per jobId SUM(cpu) ordered descending, with a HAVING."""
    rng = np.random.default_rng(3)
    n = 300_000
    cols = [rng.integers(0, 60000, n, dtype=np.int64), rng.integers(-500, 500, n, dtype=np.int64),
            rng.integers(0, 100, n, dtype=np.int32)]
    aggs = [(SUM, 2), (COUNT, 0)]
    got, cnt, status = gpu_query(lms, cols, [(1, 0, 0)], lms.Window(0, 60000, 10000, 0), aggs,
                                 having=(1, GE, 40), order=(0, True))
    assert status == 0
    exp = oracle.window_query(cols, [1], 0, 60000, 10000, 0, aggs, having=(1, GE, 40), order_by=(0, True))
    assert cnt == len(exp["wstart"]) > 0
    assert_query_equal(got, exp, aggs, True, "single key ordered")


def test_equality_filter_cm2s(lms):
    """CM2S: eventType == 1, AVG(cpu) per category over a sliding window."""
    rng = np.random.default_rng(4)
    n = 250_000
    cols = [rng.integers(0, 60000, n, dtype=np.int64), rng.integers(0, 12, n, dtype=np.int32),
            rng.integers(0, 4, n, dtype=np.int32), rng.random(n).astype(np.float32)]
    aggs = [(AVG, 3), (COUNT, 0)]
    preds = [(2, EQ, 1)]
    w = lms.Window(0, 60000, 5000, 0)
    got, cnt, status = gpu_query(lms, cols, [(1, 0, 0)], w, aggs, preds=preds)
    assert status == 0
    exp = oracle.window_query(cols, [1], 0, 60000, 5000, 0, aggs, preds=preds)
    assert cnt == len(exp["wstart"])
    assert_query_equal(got, exp, aggs, False, "cm2s")
    # the same through the single-key operator
    g, d = lms.lms_window_agg(to_dev(cols), 1, w, aggs, preds)
    torch.cuda.synchronize()
    assert [int(x) for x in d.cpu()] == [cnt, 0]


def test_query_errors_on_device(lms):
    cols = lr_cols(6, 50_000)
    aggs = [(COUNT, 0)]
    w = lms.Window(0, 1000, 0, 0)
    # a key outside its declared domain
    got, cnt, status = gpu_query(lms, cols, [(1, 0, 8), (2, 0, 1)], w, aggs)
    assert status == lms.LMS_ERANGE
    # capacity below the groups before HAVING
    got, cnt, status = gpu_query(lms, cols, KEYS, w, aggs, cap=100, having=(0, GE, 1 << 30))
    assert status == lms.LMS_ECAPACITY
    # an empty batch
    empty = [c[:0] for c in cols]
    got, cnt, status = gpu_query(lms, empty, KEYS, w, aggs, cap=16)
    assert (cnt, status) == (0, 0)


def gpu_self_join(lms, cols, key_col, window, preds=(), cap=None):
    (ws, l, a), d = lms.lms_window_self_join(to_dev(cols), key_col, window, preds, cap=cap)
    torch.cuda.synchronize()
    cnt, status = [int(x) for x in d.cpu()]
    m = min(cnt, ws.numel())
    ws, l, a = ws[:m].cpu().numpy(), l[:m].cpu().numpy().astype(np.int64), a[:m].cpu().numpy().astype(np.int64)
    order = np.lexsort((a, l, ws))
    return (ws[order], l[order], a[order]), cnt, status


@pytest.mark.parametrize("n,length,slide,origin,key_dt", [
    (20_000, 30000, 5000, 0, np.int64),    # LR1: range 30 s slide 5 s
    (30_000, 1000, 0, 0, np.int64),        # tumbling
    (15_000, 7000, 3000, -400, np.int32),  # slide not dividing the range, int32 keys, negative times
    (0, 1000, 500, 0, np.int64),
])
def test_window_self_join(lms, n, length, slide, origin, key_dt):
    rng = np.random.default_rng(7)
    cols = [rng.integers(-5000, 60000, n, dtype=np.int64), rng.integers(0, 3000, n).astype(key_dt),
            rng.integers(0, 10, n, dtype=np.int32)]
    preds = [(2, LT, 8)]
    w = lms.Window(0, length, slide, origin)
    log(f"self join n={n} len={length} slide={slide}")
    exp = oracle.window_self_join(cols, 1, 0, length, slide, origin, preds)
    got, cnt, status = gpu_self_join(lms, cols, 1, w, preds, cap=max(1, len(exp[0])))
    assert status == 0 and cnt == len(exp[0])
    for g, e, name in zip(got, exp, ("wstart", "l", "a")):
        np.testing.assert_array_equal(g, e, err_msg=name)


def test_window_self_join_capacity_below_count(lms):
    rng = np.random.default_rng(8)
    n = 5000
    cols = [rng.integers(0, 10000, n, dtype=np.int64), rng.integers(0, 50, n, dtype=np.int64)]
    exp = oracle.window_self_join(cols, 1, 0, 2000, 1000, 0)
    got, cnt, status = gpu_self_join(lms, cols, 1, lms.Window(0, 2000, 1000, 0), cap=1000)
    assert status == 0 and cnt == len(exp[0]) > 1000 and len(got[0]) == 1000

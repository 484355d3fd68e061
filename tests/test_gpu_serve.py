"""The serving loop on the GPU: every query's results, gathered over all its
micro-batches, equal the oracle over the whole stream -- whether the query
runs alone or in the mix with the others (overlapping on the device, with
batch boundaries chosen by admission at run time), and in the plain
fixed-trigger form."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal, log

pytestmark = pytest.mark.gpu

RATES = (0.2e6, 1.5e6)
STEP_S = 1.0
POOL = 1 << 20  # smaller than the stream: rows wrap around the pool


@pytest.fixture(scope="module")
def serve():
    from paper_2111_04289_amd import serve as s
    return s


@pytest.fixture(scope="module")
def stream(serve):
    t = serve.Traffic(RATES, STEP_S, seed=21)
    arr = t.arrivals_ms()
    data = serve.StreamData(arr, POOL)
    cols = [c.numpy() for c in data.host_cols(0, len(arr))]
    return data, cols


def run(serve, data, mode, queries, **kw):
    log(f"serve {mode} {queries} {kw}")
    eng = serve.Engine(data, mode=mode, queries=queries, collect=True, max_keys=1 << 20, **kw)
    res = eng.run(drain_s=60)
    log(str(res))
    return eng, res


def windows(eng, q):
    parts = [r for _, _, r in eng.queries[q].results]
    nagg = len(parts[0]) - 2
    return {"key": np.concatenate([p[0] for p in parts]), "wstart": np.concatenate([p[1] for p in parts]),
            "aggs": [np.concatenate([p[2 + k] for p in parts]) for k in range(nagg)]}


def check_fp(eng, cols):
    parts = sorted(eng.queries["fp"].results, key=lambda r: r[0])
    got = [np.concatenate([p[2][j] for p in parts]) for j in range(3)]
    exp = oracle.filter_project(cols[:3], [(2, oracle.LT, 314573)], [0, 1], [(2, 2, 0)])
    for j in range(3):
        np.testing.assert_array_equal(got[j], exp[j])


def check_join(eng, data, cols):
    idx, pay = [], []
    for d0, d1, (i, p) in eng.queries["join"].results:
        idx.append(i.view(np.uint32).astype(np.int64) + d0 * data.ds_rows)
        pay.append(p)
    idx, pay = np.concatenate(idx), np.concatenate(pay)
    bk, bp = eng.bk.numpy(), eng.bp.numpy()
    ei, ep = oracle.hash_join(bk, bp, cols[1])
    o1, o2 = np.lexsort((pay, idx)), np.lexsort((ep, ei))
    np.testing.assert_array_equal(idx[o1], ei[o2])
    np.testing.assert_array_equal(pay[o1], ep[o2])


def test_results_alone_and_in_mix_equal_the_oracle(serve, stream):
    data, cols = stream
    from paper_2111_04289_amd import serve as s
    slide_exp = oracle.window_agg(cols, 1, 0, 10000, 1000, 0, s.SLIDE_AGGS, [(2, oracle.LT, 314573)])
    tumble_exp = oracle.window_agg(cols, 1, 0, 1000, 0, 0, s.TUMBLE_AGGS)
    mix, res = run(serve, data, "served", serve.QUERIES)
    assert sum(q["batches"] for q in res["queries"].values()) > 8
    alone, _ = run(serve, data, "served", ("slide",))
    alone_t, _ = run(serve, data, "served", ("tumble",))
    for name, eng in (("mix", mix), ("alone", alone)):
        assert_window_equal(windows(eng, "slide"), slide_exp, s.SLIDE_AGGS, f"slide {name}")
    for name, eng in (("mix", mix), ("alone", alone_t)):
        assert_window_equal(windows(eng, "tumble"), tumble_exp, s.TUMBLE_AGGS, f"tumble {name}")
    check_fp(mix, cols)
    check_join(mix, data, cols)
    info = mix.queries["slide"].state.info()
    assert info["late_rows"] == 0 and info["dropped_rows"] == 0
    # the overhead breakdown: shares of buffering, admission, MapDevice,
    # processing and optimizer blocking, which sum to 100 %
    for q, v in res["queries"].items():
        bd = v["breakdown_pct"]
        assert set(bd) == {"buffering", "construct_micro_batch", "map_device", "processing",
                           "optimization_blocking"}, q
        assert abs(sum(bd.values()) - 100.0) < 0.01 and bd["processing"] > 0 and bd["buffering"] > 0, (q, bd)
        assert bd["construct_micro_batch"] > 0 and bd["map_device"] >= 0 and bd["optimization_blocking"] == 0, (q, bd)


def test_plain_trigger_form_and_cpu_placement(serve, stream):
    data, cols = stream
    from paper_2111_04289_amd import serve as s
    base, res = run(serve, data, "baseline", serve.QUERIES)
    assert res["queries"]["fp"]["cpu_batches"] == 0
    slide_exp = oracle.window_agg(cols, 1, 0, 10000, 1000, 0, s.SLIDE_AGGS, [(2, oracle.LT, 314573)])
    assert_window_equal(windows(base, "slide"), slide_exp, s.SLIDE_AGGS, "slide baseline")
    check_fp(base, cols)
    check_join(base, data, cols)
    # a deadline short enough for tiny batches, so MapDevice puts some on the CPU
    small, res = run(serve, data, "served", ("fp", "join"), bound_ms=30.0)
    assert res["queries"]["fp"]["cpu_batches"] > 0 or res["queries"]["join"]["cpu_batches"] > 0
    check_fp(small, cols)
    check_join(small, data, cols)


def test_admission_waits_for_hbm(serve, stream):
    data, cols = stream
    from paper_2111_04289_amd import serve as s
    # a budget that holds any one sliding batch (its inputs and the emitted
    # windows it reserves) but never a tumbling batch beside it: both controllers
    # admit their first batch at the same poll, so one of them must wait
    budget = (1 << 20) * s.MAX_EMIT_WINDOWS * 56 + len(cols[0]) * 24 + (1 << 20)
    eng, res = run(serve, data, "served", ("slide", "tumble"), hbm_budget=budget, slots=3)
    assert res["hbm_waits"] > 0
    slide_exp = oracle.window_agg(cols, 1, 0, 10000, 1000, 0, s.SLIDE_AGGS, [(2, oracle.LT, 314573)])
    assert_window_equal(windows(eng, "slide"), slide_exp, s.SLIDE_AGGS, "slide under an HBM budget")
    tumble_exp = oracle.window_agg(cols, 1, 0, 1000, 0, 0, s.TUMBLE_AGGS)
    assert_window_equal(windows(eng, "tumble"), tumble_exp, s.TUMBLE_AGGS, "tumble under an HBM budget")

"""GPU parity of the batched tumbling query with its projection (val < 500,
v2 = 2 * val, key x 1 s tumbling, COUNT and SUM(v2)) on the uneven stream's
own batches, and of int32 projections that wrap, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal, gpu_window_agg, log, to_dev
from oracle import COUNT, GE, LT, MAX, MIN, SUM
from paper_2111_04289_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def multi_results(groups, d, b):
    cnt, status = [int(x) for x in d[b].cpu()]
    g = groups[b]
    m = min(cnt, g.cap)
    return {"key": g.key[:m].cpu().numpy(), "wstart": g.wstart[:m].cpu().numpy(),
            "aggs": [a[:m].cpu().numpy() for a in g.aggs]}, cnt, status


def test_batched_stream_query_with_projection(lms):
    """Sixteen batches of the uneven stream (two of at least 2^22 rows) in one
    persistent launch per stage under the packaged batched tuning, eager and
    replayed from a graph: every batch equals the oracle."""
    from paper_2111_04289_amd import autotune
    sizes = [int(s) for s in datagen.stream_batch_sizes()[:14]] + [1 << 22, (1 << 22) + 4321]
    log(f"batched stream query sizes={sizes}")
    batches = [datagen.stream_batch(b, n) for b, n in enumerate(sizes)]
    preds, projs = [(2, LT, 500)], [(2, 2, 0)]
    aggs = [(COUNT, 0), (SUM, 4)]
    w = lms.Window(0, 1000, 0, 0)
    exps = [oracle.window_agg(c, 1, 0, 1000, 0, 0, aggs, preds, projs) for c in batches]
    tuned = autotune.apply("batched")
    assert tuned, "packaged batched tuning missing"
    try:
        dev = [to_dev(c) for c in batches]
        job = lms.MultiJob(1, w, aggs, preds, projs)
        groups, d = job.prepare(dev)
        job.freeze()
        job.launch()
        torch.cuda.synchronize()
        for b in range(len(batches)):
            got, cnt, status = multi_results(groups, d, b)
            assert status == 0 and cnt == len(exps[b]["key"]), f"batch {b}"
            assert_window_equal(got, exps[b], aggs, f"eager batch {b}")
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            job.launch()
        for rep in range(2):
            d.fill_(-7)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            for b in range(len(batches)):
                got, cnt, status = multi_results(groups, d, b)
                assert status == 0, f"replay {rep} batch {b}"
                assert_window_equal(got, exps[b], aggs, f"replay {rep} batch {b}")
        del graph
    finally:
        lms.set_tuning()


def wrap_cols(seed, n):
    rng = np.random.default_rng(seed)
    ts = rng.integers(0, 20000, n, dtype=np.int64)
    key = rng.integers(0, 300, n, dtype=np.int64)
    val = rng.integers(1 << 30, (1 << 31) - 1, n, dtype=np.int32)  # 3 * val wraps modulo 2^32
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


def test_filter_project_int32_wrap(lms):
    cols = wrap_cols(1, 200000)
    preds = [(2, GE, (1 << 30) + (1 << 28))]
    projs = [(2, 3, 0), (2, -5, 7), (0, (1 << 50) + 1, 3)]
    out, d = lms.lms_filter_project(to_dev(cols), preds, [1, 2], projs)
    torch.cuda.synchronize()
    m, status = [int(x) for x in d.cpu()]
    exp = oracle.filter_project(cols, preds, [1, 2], projs)
    assert status == 0 and m == len(exp[0])
    for j in range(len(exp)):
        np.testing.assert_array_equal(out[j][:m].cpu().numpy(), exp[j], err_msg=f"column {j}")
    # the projection did wrap: int32 results differ from the exact products
    exact = 3 * exp[1].astype(np.int64)
    assert (exp[2].astype(np.int64) != exact).any()


@pytest.mark.parametrize("length,slide", [(1000, 0), (3000, 1000)])
def test_window_agg_over_wrapping_projection(lms, length, slide):
    cols = wrap_cols(2, 300000)
    # 3 * val modulo 2^32 is negative for val in [1.25, 4/3) * 2^30 and
    # positive above, so both signs of wrapped value reach the aggregates
    preds = [(2, GE, (1 << 30) + (1 << 28))]
    projs = [(2, 3, 0)]
    aggs = [(COUNT, 0), (SUM, 4), (MIN, 4), (MAX, 4)]
    got, cnt, status = gpu_window_agg(cols, 1, 0, length, slide, 0, aggs, preds, projs)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, length, slide, 0, aggs, preds, projs)
    assert_window_equal(got, exp, aggs, "wrap")
    assert (exp["aggs"][2] < 0).any() and (exp["aggs"][3] > 0).any()  # both signs wrapped
    log("multi-batch form of the same query")
    batches = [wrap_cols(10 + i, n) for i, n in enumerate([1000, 77777, 5, 150000])]
    w = lms.Window(0, length, slide, 0)
    groups, d, _ = lms.lms_window_agg_multi([to_dev(c) for c in batches], 1, w, aggs, preds, projs)
    torch.cuda.synchronize()
    for b, c in enumerate(batches):
        g, n, st = multi_results(groups, d, b)
        assert st == 0
        assert_window_equal(g, oracle.window_agg(c, 1, 0, length, slide, 0, aggs, preds, projs), aggs, f"multi {b}")

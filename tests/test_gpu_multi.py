"""GPU parity of the multi-batch windowed group-by (one persistent launch per
stage over many micro-batches) against the CPU oracle, batch by batch, and of
its graph-captured launch replayed after new data and new descriptors."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal, log, to_dev
from oracle import AVG, COUNT, LT, MAX, MIN, SUM
from paper_2111_04289_amd import datagen

pytestmark = pytest.mark.gpu

AGGS = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3)]
PREDS = [(2, LT, 600)]


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def batch_cols(seed, n, nkeys=400, tspan=20000):
    rng = np.random.default_rng(seed)
    ts = np.sort(rng.integers(0, tspan, n, dtype=np.int64))
    key = datagen.splitmix64(rng.integers(0, nkeys, n).astype(np.uint64)).view(np.int64)
    val = rng.integers(-1000, 1000, n, dtype=np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


def result(groups, d, b):
    cnt, status = [int(x) for x in d[b].cpu()]
    g = groups[b]
    m = min(cnt, g.cap)
    return {"key": g.key[:m].cpu().numpy(), "wstart": g.wstart[:m].cpu().numpy(),
            "aggs": [a[:m].cpu().numpy() for a in g.aggs]}, cnt, status


def check_all(lms, batches, groups, d, window, what):
    torch.cuda.synchronize()
    for b, cols in enumerate(batches):
        got, cnt, status = result(groups, d, b)
        assert status == 0, f"{what} batch {b}: status {status}"
        exp = oracle.window_agg(cols, 1, 0, window.length, window.slide, window.origin, AGGS, PREDS)
        assert cnt == len(exp["key"]), f"{what} batch {b}"
        assert_window_equal(got, exp, AGGS, f"{what} batch {b}")


SIZES = [0, 1, 5, 777, 4096, 4097, 30000, 70001, 3, 150000, 12345, 2]


@pytest.mark.parametrize("length,slide", [(1000, 0), (3000, 500)])
def test_multi_matches_oracle(lms, length, slide):
    log(f"multi sizes={SIZES} window={length}/{slide}")
    batches = [batch_cols(100 + i, n) for i, n in enumerate(SIZES)]
    w = lms.Window(0, length, slide, 0)
    groups, d, job = lms.lms_window_agg_multi([to_dev(c) for c in batches], 1, w, AGGS, PREDS)
    check_all(lms, batches, groups, d, w, "multi")


@pytest.mark.parametrize("aggs", [
    [(COUNT, 0), (SUM, 4), (MIN, 4), (MAX, 2), (AVG, 5), (AVG, 3)],  # five accumulators
    [(SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3), (SUM, 4), (MIN, 4), (MAX, 4), (AVG, 5)],  # eight, the widest
])
def test_multi_wide_value_columns(lms, aggs):
    """The persistent launch on batches with int64 and float64 value columns
    next to int32 and float32 ones (staged records with 8-byte values ahead
    of the pane), each batch against the oracle."""
    batches = []
    for i, n in enumerate([50000, 1, 120001, 777]):
        rng = np.random.default_rng(300 + i)
        ts = rng.integers(0, 20000, n, dtype=np.int64)
        key = rng.integers(0, 900, n, dtype=np.int64)
        val = rng.integers(-1000, 1000, n, dtype=np.int32)
        f = rng.standard_normal(n).astype(np.float32)
        v64 = rng.integers(-(1 << 40), 1 << 40, n, dtype=np.int64)
        f64 = rng.standard_normal(n) * 1e6
        batches.append([ts, key, val, f, v64, f64])
    w = lms.Window(0, 3000, 1000, 0)
    log(f"multi wide values aggs={aggs}")
    groups, d, _ = lms.lms_window_agg_multi([to_dev(c) for c in batches], 1, w, aggs, PREDS)
    torch.cuda.synchronize()
    for b, cols in enumerate(batches):
        got, cnt, status = result(groups, d, b)
        assert status == 0, f"wide batch {b}: status {status}"
        exp = oracle.window_agg(cols, 1, 0, w.length, w.slide, w.origin, aggs, PREDS)
        assert cnt == len(exp["key"]), f"wide batch {b}"
        assert_window_equal(got, exp, aggs, f"wide batch {b}")


def test_multi_equals_single_calls(lms):
    log("multi vs single")
    batches = [batch_cols(200 + i, n) for i, n in enumerate([9000, 40000, 1, 65536])]
    w = lms.Window(0, 2000, 1000, 0)
    dev = [to_dev(c) for c in batches]
    groups, d, _ = lms.lms_window_agg_multi(dev, 1, w, AGGS, PREDS)
    torch.cuda.synchronize()
    for b in range(len(batches)):
        g1, d1 = lms.lms_window_agg(dev[b], 1, w, AGGS, PREDS)
        torch.cuda.synchronize()
        single = {"key": g1.key[:int(d1[0])].cpu().numpy(), "wstart": g1.wstart[:int(d1[0])].cpu().numpy(),
                  "aggs": [a[:int(d1[0])].cpu().numpy() for a in g1.aggs]}
        got, cnt, status = result(groups, d, b)
        assert status == 0 and cnt == int(d1[0])
        assert_window_equal(got, single, AGGS, f"multi vs single batch {b}")


def test_multi_graph_replay(lms):
    """Capture the launch once; replay it after eager work, after new data in
    the same buffers, after a new prepare, and on a job too large for it."""
    sizes = [5000, 20000, 333, 60000]
    w = lms.Window(0, 3000, 1000, 0)
    batches = [batch_cols(300 + i, n) for i, n in enumerate(sizes)]
    dev = [to_dev(c) for c in batches]
    job = lms.MultiJob(1, w, AGGS, PREDS)
    big = [batch_cols(600, 1200000)]  # more partitions than any batch above (128 against 32)
    dbig = [to_dev(c) for c in big]
    job.reserve(job.workspace_bytes(dbig))  # the captured graph reads this workspace, so it never moves
    groups, d = job.prepare(dev)
    job.freeze(max_nparts=16)
    job.launch()  # eager run: sets kernel attributes before capture
    check_all(lms, batches, groups, d, w, "eager")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        job.launch()
    for rep in range(3):
        log(f"graph replay {rep}: new data in the same buffers")
        batches = [batch_cols(400 + 10 * rep + i, n) for i, n in enumerate(sizes)]
        for t, c in zip(dev, batches):
            for td, cn in zip(t, c):
                td.copy_(torch.from_numpy(cn))
        torch.cuda.synchronize()
        _ = (dev[0][2] * 3).sum().item()  # unrelated eager work between replays
        graph.replay()
        check_all(lms, batches, groups, d, w, f"replay {rep}")
    log("graph replay after a new prepare with other sizes")
    sizes2 = [100, 7000, 0, 45000, 12]
    batches2 = [batch_cols(500 + i, n) for i, n in enumerate(sizes2)]
    dev2 = [to_dev(c) for c in batches2]
    groups2, d2 = job.prepare(dev2)
    assert job.cfg.max_nparts <= job.launch_cfg.max_nparts and job.cfg.ma == job.launch_cfg.ma
    graph.replay()
    check_all(lms, batches2, groups2, d2, w, "replay after prepare")
    log("graph replay on a job beyond the captured limits is rejected")
    ws_ptr = job.ws.data_ptr()
    g3, d3 = job.prepare(dbig)
    assert job.ws.data_ptr() == ws_ptr
    assert job.cfg.max_nparts > job.launch_cfg.max_nparts
    graph.replay()
    torch.cuda.synchronize()
    assert int(d3[0][1]) == lms.LMS_EINVAL and int(d3[0][0]) == 0


@pytest.mark.parametrize("tuning", [dict(chunk_rows=2048, part_rows=8192, piece_rows=1024, grid_per_cu=1,
                                         lds_groups=1024),
                                    dict(chunk_rows=65536, part_rows=65536, piece_rows=32768, grid_per_cu=8)])
def test_tuning_keeps_results(lms, tuning):
    """Tile and schedule parameters change the work split, never the result."""
    log(f"tuning {tuning}")
    lms.set_tuning(**tuning)
    try:
        cols = batch_cols(700, 200000, nkeys=5000)
        w = lms.Window(0, 3000, 1000, 0)
        g, d = lms.lms_window_agg(to_dev(cols), 1, w, AGGS, PREDS)
        check_all(lms, [cols], [g], d.view(1, 2), w, f"single {tuning}")
        batches = [batch_cols(710 + i, n) for i, n in enumerate(SIZES)]
        groups, dm, _ = lms.lms_window_agg_multi([to_dev(c) for c in batches], 1, w, AGGS, PREDS)
        check_all(lms, batches, groups, dm, w, f"multi {tuning}")
    finally:
        lms.set_tuning()

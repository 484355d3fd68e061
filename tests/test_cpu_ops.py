"""The CPU execution functions (the CPU side of MapDevice) against the oracle.
They run on host memory, so these tests need no GPU."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal
from paper_2111_04289_amd import datagen

lms = pytest.importorskip("paper_2111_04289_amd.lms")

AGGS = [(oracle.COUNT, 0), (oracle.SUM, 2), (oracle.MIN, 2), (oracle.MAX, 2), (oracle.AVG, 3), (oracle.SUM, 4)]


def cols_np(seed, n, nkeys, tspan, neg=False):
    rng = np.random.default_rng(seed)
    ts = rng.integers(-tspan if neg else 0, tspan, n, dtype=np.int64)
    key = datagen.splitmix64(rng.integers(0, nkeys, n).astype(np.uint64)).view(np.int64)
    val = rng.integers(-500, 500, n, dtype=np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


@pytest.mark.parametrize("n,length,slide,origin,threads", [(0, 10, 2, 0, 2), (1, 10, 0, 0, 1),
                                                            (5000, 100, 30, 7, 1), (20000, 1000, 250, -3, 4),
                                                            (30000, 60, 60, 0, 3)])
def test_cpu_window_agg_matches_oracle(n, length, slide, origin, threads):
    c = cols_np(n + threads, n, 300, 5000, neg=True)
    preds, projs = [(2, oracle.LT, 200)], [(2, 3, 1)]
    k, ws, aggs, cnt = lms.lms_cpu_window_agg([torch.from_numpy(x) for x in c], 1, lms.Window(0, length, slide, origin),
                                              AGGS, preds, projs, nthreads=threads)
    got = {"key": k.numpy(), "wstart": ws.numpy(), "aggs": [a.numpy() for a in aggs]}
    exp = oracle.window_agg(c, 1, 0, length, slide, origin, AGGS, preds, projs)
    assert cnt == len(exp["key"])
    assert_window_equal(got, exp, AGGS, "cpu")


def test_cpu_window_agg_config0():
    c = datagen.config0()
    aggs = [(oracle.COUNT, 0), (oracle.SUM, 4)]
    k, ws, a, cnt = lms.lms_cpu_window_agg([torch.from_numpy(x) for x in c], 1, lms.Window(0, 1000, 0, 0), aggs,
                                           [(2, oracle.LT, 500)], [(2, 2, 0)], nthreads=4)
    exp = oracle.window_agg(c, 1, 0, 1000, 0, 0, aggs, [(2, oracle.LT, 500)], [(2, 2, 0)])
    assert_window_equal({"key": k.numpy(), "wstart": ws.numpy(), "aggs": [x.numpy() for x in a]}, exp, aggs, "c0")


@pytest.mark.parametrize("threads", [1, 4])
def test_cpu_filter_project_matches_oracle(threads):
    c = cols_np(3, 40001, 50, 1000)
    preds, keep, projs = [(2, oracle.GE, -100), (3, oracle.LT, 0, 0.7)], [0, 1, 3], [(2, 2, 0)]
    out = lms.lms_cpu_filter_project([torch.from_numpy(x) for x in c], preds, keep, projs, nthreads=threads)
    exp = oracle.filter_project(c, preds, keep, projs)
    for j in range(4):
        np.testing.assert_array_equal(out[j].numpy(), exp[j])


@pytest.mark.parametrize("dup,threads", [(False, 1), (True, 4)])
def test_cpu_hash_join_matches_oracle(dup, threads):
    bk, bp = (datagen.static_table_dup(5000, 3000) if dup else datagen.static_table(5000))
    pk = datagen.zipf_keys(np.random.default_rng(2), 30000, 1.1, 5000)
    i, p, cnt = lms.lms_cpu_hash_join(torch.from_numpy(bk), torch.from_numpy(bp), torch.from_numpy(pk),
                                      cap=200000, nthreads=threads)
    ei, ep = oracle.hash_join(bk, bp, pk)
    assert cnt == len(ei)
    np.testing.assert_array_equal(i.numpy().astype(np.int64), ei)
    o1, o2 = np.lexsort((p.numpy(), i.numpy())), np.lexsort((ep, ei))
    np.testing.assert_array_equal(p.numpy()[o1], ep[o2])

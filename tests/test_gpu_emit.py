"""Re-emission of a windowed group-by from its intact workspace
(lms_window_agg_emit), through the C-ABI binding, against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal, log, to_dev
from oracle import AVG, COUNT, MAX, MIN, SUM
from paper_2111_04289_amd import datagen

pytestmark = pytest.mark.gpu

AGGS5 = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3)]


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def fetch(g, d):
    torch.cuda.synchronize()
    cnt, status = [int(x) for x in d.cpu()]
    m = min(cnt, g.cap)
    res = {"key": g.key[:m].cpu().numpy(), "wstart": g.wstart[:m].cpu().numpy(),
           "aggs": [a[:m].cpu().numpy() for a in g.aggs]}
    return res, cnt, status


def zipf_cols(seed, n, tspan):
    rng = np.random.default_rng(seed)
    ts = rng.integers(0, tspan, n, dtype=np.int64)
    key = datagen.zipf_keys(rng, n, 1.1, 1 << 16)
    val = rng.integers(-1000, 1000, n, dtype=np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


@pytest.mark.parametrize("n,length,slide", [(1 << 20, 10000, 1000), (300000, 1000, 0), (5000, 300, 100)])
def test_emit_after_short_capacity_gives_every_group(lms, n, length, slide):
    """First call with a third of the needed capacity, then re-emit with the
    full count: equal to the oracle (Zipf keys: split partitions included)."""
    log(f"emit n={n} len={length} slide={slide}")
    cols = zipf_cols(n + length, n, 60000)
    exp = oracle.window_agg(cols, 1, 0, length, slide, 0, AGGS5, [(2, oracle.LT, 500)])
    total = len(exp["key"])
    dc = to_dev(cols)
    ws = lms.Workspace(dc[0].device)
    w = lms.Window(0, length, slide, 0)
    g, d = lms.lms_window_agg(dc, 1, w, AGGS5, [(2, lms.LT, 500)], cap=max(1, total // 3), workspace=ws)
    _, cnt, status = fetch(g, d)
    assert (cnt, status) == (total, 0)
    del dc  # the input is not needed for the re-emission
    torch.cuda.synchronize()
    g2, d2 = lms.lms_window_agg_emit(AGGS5, ws, cap=cnt)
    got, cnt2, status2 = fetch(g2, d2)
    assert (cnt2, status2) == (total, 0)
    assert_window_equal(got, exp, AGGS5, "re-emitted")
    # and once more, into the same outputs
    g3, d3 = lms.lms_window_agg_emit(AGGS5, ws, groups=g2)
    got3, cnt3, status3 = fetch(g3, d3)
    assert (cnt3, status3) == (total, 0)
    assert_window_equal(got3, exp, AGGS5, "emitted twice")


def test_emit_after_empty_batch(lms):
    cols = [np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32)]
    dc = to_dev(cols)
    ws = lms.Workspace(torch.device("cuda"))
    g, d = lms.lms_window_agg(dc, 1, lms.Window(0, 100, 0, 0), AGGS5, cap=4, workspace=ws)
    assert fetch(g, d)[1:] == (0, 0)
    g2, d2 = lms.lms_window_agg_emit(AGGS5, ws, cap=4)
    assert fetch(g2, d2)[1:] == (0, 0)


def test_emit_rejects_unfilled_workspace_and_other_aggregates(lms):
    ws = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    g, d = lms.lms_window_agg_emit(AGGS5, ws, cap=4)
    assert fetch(g, d)[2] == lms.LMS_EINVAL
    cols = zipf_cols(3, 20000, 5000)
    w = lms.Workspace(torch.device("cuda"))
    g, d = lms.lms_window_agg(to_dev(cols), 1, lms.Window(0, 100, 0, 0), AGGS5, workspace=w)
    assert fetch(g, d)[2] == 0
    g2, d2 = lms.lms_window_agg_emit(AGGS5[:2], w, cap=10)
    assert fetch(g2, d2)[2] == lms.LMS_EINVAL
    with pytest.raises(lms.LmsError):
        lms.lms_window_agg_emit(AGGS5, torch.zeros(16, dtype=torch.uint8, device="cuda"), cap=4)

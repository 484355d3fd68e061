"""GPU parity: the HIP operators (through the C-ABI) against the CPU oracle.

Integer results must be bit-exact; AVG within 1e-5 relative.  Sizes span
several tiles, partitions and pieces with ragged tails; edge cases cover empty
inputs, empty filters, hot keys, key values equal to the table's empty marker,
LDS overflow of a partition, output capacity below the group count, a key
with more panes than one workgroup table holds, and a window spanning more.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal, gpu_window_agg, log, to_dev
from oracle import AVG, COUNT, GE, GT, LE, LT, MAX, MIN, NE, SUM
from paper_2111_04289_amd import datagen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def rand_cols(seed, n, nkeys, tspan, key64=True, neg=False, zipf=False):
    rng = np.random.default_rng(seed)
    lo = -tspan if neg else 0
    ts = rng.integers(lo, tspan, n, dtype=np.int64)
    if zipf:
        key = datagen.zipf_keys(rng, n, 1.1, nkeys)
    elif key64:
        key = datagen.splitmix64(rng.integers(0, nkeys, n).astype(np.uint64)).view(np.int64)
    else:
        key = rng.integers(0, nkeys, n, dtype=np.int32)
    val = rng.integers(-1000, 1000, n, dtype=np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


# ---------------------------------------------------------------- filter + project

@pytest.mark.parametrize("n,seed", [(0, 0), (1, 1), (4095, 2), (4097, 3), (70001, 4), (300000, 5)])
def test_filter_project_parity(lms, n, seed):
    log(f"filter_project n={n} seed={seed}")
    cols = rand_cols(seed, n, 50, 1000, neg=True)
    cols[3][::97] = np.nan
    preds = [(2, LT, 300), (3, NE, 0, 0.5)]
    keep = [0, 1, 3]
    projs = [(2, 2, 0), (0, -3, 11)]
    out, d = lms.lms_filter_project(to_dev(cols), preds, keep, projs)
    torch.cuda.synchronize()
    m, status = [int(x) for x in d.cpu()]
    assert status == 0
    exp = oracle.filter_project(cols, preds, keep, projs)
    assert m == len(exp[0])
    for j in range(len(exp)):
        g = out[j][:m].cpu().numpy()
        if g.dtype.kind == "f":
            np.testing.assert_array_equal(np.isnan(g), np.isnan(exp[j]))
            np.testing.assert_array_equal(g[~np.isnan(g)], exp[j][~np.isnan(exp[j])])
        else:
            np.testing.assert_array_equal(g, exp[j])


def _check_filter(lms, cols, dcols, preds, keep, projs):
    out, d = lms.lms_filter_project(dcols, preds, keep, projs)
    torch.cuda.synchronize()
    m, status = [int(x) for x in d.cpu()]
    assert status == 0
    exp = oracle.filter_project(cols, preds, keep, projs)
    assert m == len(exp[0])
    for j in range(len(exp)):
        g = out[j][:m].cpu().numpy()
        if g.dtype.kind == "f":
            np.testing.assert_array_equal(np.isnan(g), np.isnan(exp[j]))
            np.testing.assert_array_equal(g[~np.isnan(g)], exp[j][~np.isnan(exp[j])])
        else:
            np.testing.assert_array_equal(g, exp[j])
    return m


@pytest.mark.parametrize("n,offset", [(70001, 1), (70001, 2), (300000, 3)])
def test_filter_project_unaligned_columns(lms, n, offset):
    """Columns that do not start on a 16-byte boundary (views one or more rows
    into a buffer) take the row-by-row loads; results must not change."""
    log(f"filter_project unaligned n={n} offset={offset}")
    full = rand_cols(11, n + offset, 50, 1000, neg=True)
    cols = [c[offset:] for c in full]
    dcols = [c[offset:] for c in to_dev(full)]
    assert any(c.data_ptr() % 16 for c in dcols)
    _check_filter(lms, cols, dcols, [(2, LT, 300), (3, NE, 0, 0.5)], [0, 1, 3], [(2, 2, 0), (0, -3, 11)])


def test_filter_project_sparse_and_dense_tiles(lms):
    """A predicate on the sorted time column passes every row of some tiles, a
    few rows of others and none of the rest: dense tiles use the quad loads,
    sparse ones the passing rows' loads, in one launch."""
    n = 200003
    cols = rand_cols(12, n, 50, 1000, neg=True)
    cols[0] = np.sort(cols[0])
    cols[0][n // 2:n // 2 + 9000:97] = -2000  # scattered passing rows in the upper half
    m = _check_filter(lms, cols, to_dev(cols), [(0, LT, -500)], [0, 1, 2, 3], [(1, 7, -1)])
    assert 0 < m < n


def test_filter_project_all_and_none(lms):
    cols = rand_cols(9, 10000, 10, 100)
    for preds, expect in [([], 10000), ([(2, GE, 5000)], 0), ([(2, LE, 5000)], 10000)]:
        out, d = lms.lms_filter_project(to_dev(cols), preds, [0, 2], [])
        torch.cuda.synchronize()
        assert int(d[0]) == expect
        if expect:
            np.testing.assert_array_equal(out[1][:expect].cpu().numpy(), cols[2])


def test_filter_project_wide_columns(lms):
    """Predicates on a float64 (with NaNs) and an int64 column, float64 and
    int64 columns kept, and an int64 projection that wraps: the 8-byte paths
    of the predicate, the copy and the projection."""
    n = 150001
    cols = wide_value_cols(51, n)
    cols[5][::89] = np.nan
    log("filter_project wide columns")
    m = _check_filter(lms, cols, to_dev(cols), [(5, GT, 0, -2e5), (4, LT, 1 << 39)], [0, 5, 4, 3],
                      [(4, 1 << 30, 7), (2, -5, 1)])
    assert 0 < m < n


# ---------------------------------------------------------------- windowed group-by

AGGS5 = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3)]


def test_config0_tumbling_exact():
    cols = datagen.config0()
    aggs = [(COUNT, 0), (SUM, 4)]
    preds, projs = [(2, LT, 500)], [(2, 2, 0)]
    log("config0 tumbling")
    got, cnt, status = gpu_window_agg(cols, 1, 0, 1000, 0, 0, aggs, preds, projs)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, 1000, 0, 0, aggs, preds, projs)
    assert cnt == len(exp["key"])
    assert_window_equal(got, exp, aggs, "config0")


@pytest.mark.parametrize("length,slide", [(1000, 0), (3000, 1000)])
def test_window_agg_graph_replay(lms, length, slide):
    """One call captured in a HIP graph (the plan is fixed by the batch size at
    capture) and replayed on new data in the same input buffers, with eager
    work between replays: every replay equals the oracle on its data."""
    n = 65536
    aggs = [(COUNT, 0), (SUM, 4), (MIN, 2), (AVG, 3)]
    preds, projs = [(2, LT, 500)], [(2, 2, 0)]
    w = lms.Window(0, length, slide, 0)
    dev = to_dev(datagen.config0(n))
    groups = lms.Groups(n * 3, aggs, dev[0].device)
    d = torch.zeros(2, dtype=torch.int64, device=dev[0].device)
    ws = lms.Workspace(dev[0].device)

    def call():
        lms.lms_window_agg(dev, 1, w, aggs, preds, projs, groups=groups, d_count=d, workspace=ws)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        call()  # sizes the workspace and sets kernel attributes before capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for rep in range(4):
        log(f"window_agg graph replay {rep} len={length} slide={slide}")
        cols = rand_cols(700 + rep, n, 1024, 10000, key64=False)  # the dtypes of the captured batch
        for t, c in zip(dev, cols):
            t.copy_(torch.from_numpy(c))
        d.fill_(-1)
        _ = (dev[2] * 3).sum().item()  # unrelated eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        cnt, status = [int(x) for x in d.cpu()]
        assert status == 0
        got = {"key": groups.key[:cnt].cpu().numpy(), "wstart": groups.wstart[:cnt].cpu().numpy(),
               "aggs": [a[:cnt].cpu().numpy() for a in groups.aggs]}
        exp = oracle.window_agg(cols, 1, 0, length, slide, 0, aggs, preds, projs)
        assert cnt == len(exp["key"]) > 0
        assert_window_equal(got, exp, aggs, f"graph replay {rep}")


@pytest.mark.parametrize("n,length,slide,origin,key64,neg,nkeys,tspan", [
    (1, 10, 0, 0, True, False, 5, 100),
    (1000, 10, 3, 5, True, True, 7, 200),
    (50000, 10000, 1000, 0, True, False, 3000, 60000),
    (123457, 3000, 1000, -250, False, True, 500, 20000),
    (200003, 1000, 400, 17, True, False, 20000, 30000),
    (65536, 7, 7, 0, False, False, 1024, 10000),
    (300000, 60, 5, 3, True, True, 100000, 3000),
])
def test_window_agg_parity(n, length, slide, origin, key64, neg, nkeys, tspan):
    log(f"window_agg n={n} L={length} S={slide} origin={origin}")
    cols = rand_cols(n, n, nkeys, tspan, key64=key64, neg=neg)
    preds = [(2, LT, 600)]
    projs = [(2, 3, -7)]
    aggs = AGGS5 + [(SUM, 4), (MIN, 4)]
    got, cnt, status = gpu_window_agg(cols, 1, 0, length, slide, origin, aggs, preds, projs)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, length, slide, origin, aggs, preds, projs)
    assert cnt == len(exp["key"])
    assert_window_equal(got, exp, aggs, f"n={n}")


@pytest.mark.parametrize("n", [131072, 131073])
@pytest.mark.parametrize("length,slide", [(1000, 0), (5000, 1000)])
def test_window_agg_scan_paths_at_the_chunk_threshold(n, length, slide):
    """64 chunks of 2048 rows take the one-workgroup scans, 65 chunks the three
    scan launches; both against the oracle."""
    log(f"scan paths n={n} len={length} slide={slide}")
    cols = rand_cols(n % 7, n, 3000, 20000)
    preds, projs = [(2, LT, 300)], [(2, 3, -7)]
    aggs = [(COUNT, 0), (SUM, 4), (MAX, 2), (AVG, 3)]
    got, cnt, status = gpu_window_agg(cols, 1, 0, length, slide, 0, aggs, preds, projs)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, length, slide, 0, aggs, preds, projs)
    assert cnt == len(exp["key"]) > 0
    assert_window_equal(got, exp, aggs, f"n={n}")

@pytest.mark.parametrize("tmax", [640, 650, 10])
def test_window_agg_pane_span_at_mask_width(tmax):
    """Panes 0..63 (span 63), 0..64 (span 64) and a single pane: the sliding
    composition ranks a key's panes with a 64-bit mask up to span 63 and by
    comparison beyond; both must give the oracle's result."""
    n = 60000
    rng = np.random.default_rng(tmax)
    cols = [rng.integers(0, tmax, n, dtype=np.int64), rng.integers(0, 300, n, dtype=np.int64),
            rng.integers(-1000, 1000, n, dtype=np.int32), rng.standard_normal(n).astype(np.float32)]
    log(f"pane span tmax={tmax}")
    got, cnt, status = gpu_window_agg(cols, 1, 0, 50, 10, 0, AGGS5)
    assert status == 0
    assert_window_equal(got, oracle.window_agg(cols, 1, 0, 50, 10, 0, AGGS5), AGGS5, f"tmax={tmax}")


@pytest.mark.parametrize("offset", [0, 1, 3])
def test_window_agg_column_views(offset):
    """Columns that are views some rows into a buffer (not on a 16-byte
    boundary unless offset is 0) take the row-by-row loads of the histogram
    and scatter passes; results must not change."""
    n = 120001
    full = rand_cols(31 + offset, n + offset, 900, 30000, neg=True)
    cols = [c[offset:] for c in full]
    dcols = [c[offset:] for c in to_dev(full)]
    log(f"window views offset={offset}")
    preds = [(2, LT, 400)]
    got, cnt, status = gpu_window_agg(cols, 1, 0, 5000, 1000, 7, AGGS5, preds, dev_cols=dcols)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, 5000, 1000, 7, AGGS5, preds)
    assert cnt == len(exp["key"])
    assert_window_equal(got, exp, AGGS5, f"offset={offset}")


def test_window_agg_eight_accumulators():
    """Eight aggregates, each with an accumulator of its own (the widest
    instantiation of the kernels), over two input columns and a projection."""
    n = 150001
    cols = rand_cols(21, n, 700, 20000, neg=True)
    aggs = [(SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3), (SUM, 4), (MIN, 4), (MAX, 4), (AVG, 2)]
    preds = [(2, LT, 500)]
    projs = [(2, 3, -7)]
    log("eight accumulators")
    got, cnt, status = gpu_window_agg(cols, 1, 0, 3000, 1000, 0, aggs, preds, projs)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, 3000, 1000, 0, aggs, preds, projs)
    assert cnt == len(exp["key"])
    assert_window_equal(got, exp, aggs, "eight")


def wide_value_cols(seed, n, nkeys=3000):
    """ts, key, an int32 and a float32 value column, and an int64 and a
    float64 one (values below 2^40, so no sum wraps)."""
    rng = np.random.default_rng(seed)
    ts = rng.integers(0, 30000, n, dtype=np.int64)
    key = rng.integers(0, nkeys, n, dtype=np.int64)
    v32 = rng.integers(-1000, 1000, n, dtype=np.int32)
    f32 = rng.standard_normal(n).astype(np.float32)
    v64 = rng.integers(-(1 << 40), 1 << 40, n, dtype=np.int64)
    f64 = rng.standard_normal(n) * 1e6
    return [ts, key, v32, f32, v64, f64]


@pytest.mark.parametrize("aggs,projs,nkeys", [
    # six accumulators: two 8-byte values ahead of the pane in the staged
    # record, two 4-byte ones behind it (a 40-byte record)
    ([(COUNT, 0), (SUM, 4), (MIN, 4), (MAX, 4), (AVG, 5), (SUM, 2), (AVG, 3)], [], 3000),
    # four accumulators over 8-byte values only, one of them a projection of
    # the int64 column (an int64 result)
    ([(SUM, 6), (AVG, 5), (MAX, 4), (COUNT, 0)], [(4, 3, 1)], 3000),
    # an 8-byte value between 4-byte ones in the aggregate order
    ([(MIN, 2), (MAX, 4), (AVG, 3)], [], 3000),
    # five keys: partitions beyond the piece size, aggregated in pieces and merged
    ([(COUNT, 0), (SUM, 4), (MIN, 4), (AVG, 5), (MAX, 2)], [], 5),
])
def test_window_agg_wide_value_columns(aggs, projs, nkeys):
    """Value columns of every width in one call: int64 and float64 values sit
    ahead of the pane in a staged record and int32 and float32 ones behind
    it, so each field of the record is read at its own word and half."""
    n = 200003
    cols = wide_value_cols(41, n, nkeys)
    cols[5][::101] = np.nan
    preds = [(2, LT, 600), (5, GT, 0, -1.5e6)]  # and a float64 predicate (NaN rows fail it)
    log(f"wide values aggs={aggs} projs={projs} nkeys={nkeys}")
    got, cnt, status = gpu_window_agg(cols, 1, 0, 5000, 1000, 0, aggs, preds, projs)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, 5000, 1000, 0, aggs, preds, projs)
    assert cnt == len(exp["key"]) > 0
    assert_window_equal(got, exp, aggs, "wide values")


def test_window_agg_zipf_hot_keys_pieces_and_merge():
    # one hot key carries ~12% of the rows: its partition is split into pieces and merged
    n = 1_000_000
    cols = datagen.config1(n)
    log("zipf 1M sliding")
    preds = [(2, LT, datagen.CONFIG1_VAL_CUT)]
    got, cnt, status = gpu_window_agg(cols, 1, 0, 10000, 1000, 0, AGGS5, preds)
    assert status == 0
    exp = oracle.window_agg(cols, 1, 0, 10000, 1000, 0, AGGS5, preds)
    assert_window_equal(got, exp, AGGS5, "zipf")


def test_window_agg_single_key_many_rows():
    n = 300000
    rng = np.random.default_rng(3)
    cols = [rng.integers(0, 5000, n, dtype=np.int64), np.full(n, 42, np.int64),
            rng.integers(0, 100, n, dtype=np.int32), rng.standard_normal(n).astype(np.float32)]
    log("single key")
    for length, slide in [(1000, 0), (1000, 250)]:
        got, cnt, status = gpu_window_agg(cols, 1, 0, length, slide, 0, AGGS5)
        assert status == 0
        assert_window_equal(got, oracle.window_agg(cols, 1, 0, length, slide, 0, AGGS5), AGGS5, f"{length}/{slide}")


def test_window_agg_lds_overflow_splits_partition():
    # all-distinct keys: each partition holds far more groups than the LDS tables
    n = 400000
    rng = np.random.default_rng(4)
    cols = [rng.integers(0, 4000, n, dtype=np.int64), rng.permutation(n).astype(np.int64) * 7919 - 10**12,
            rng.integers(0, 100, n, dtype=np.int32), rng.standard_normal(n).astype(np.float32)]
    log("distinct keys")
    got, cnt, status = gpu_window_agg(cols, 1, 0, 1000, 500, 0, AGGS5)
    assert status == 0
    assert_window_equal(got, oracle.window_agg(cols, 1, 0, 1000, 500, 0, AGGS5), AGGS5, "distinct")


def test_window_agg_sentinel_and_extreme_keys():
    n = 20000
    rng = np.random.default_rng(5)
    special = np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0, -1], np.int64)
    cols = [rng.integers(-5000, 5000, n, dtype=np.int64), special[rng.integers(0, 4, n)],
            rng.integers(-2**31, 2**31 - 1, n, dtype=np.int64).astype(np.int32), rng.standard_normal(n).astype(np.float32)]
    log("sentinel keys")
    got, cnt, status = gpu_window_agg(cols, 1, 0, 300, 100, -1, AGGS5)
    assert status == 0
    assert_window_equal(got, oracle.window_agg(cols, 1, 0, 300, 100, -1, AGGS5), AGGS5, "sentinel")


def test_window_agg_empty_and_filtered_out():
    cols = rand_cols(1, 0, 5, 100)
    got, cnt, status = gpu_window_agg(cols, 1, 0, 10, 5, 0, AGGS5, cap=16)
    assert (cnt, status) == (0, 0)
    cols = rand_cols(2, 5000, 5, 100)
    got, cnt, status = gpu_window_agg(cols, 1, 0, 10, 5, 0, AGGS5, preds=[(2, GE, 10**6)], cap=16)
    assert (cnt, status) == (0, 0)


def test_window_agg_capacity_below_count():
    cols = rand_cols(6, 50000, 300, 5000)
    exp = oracle.window_agg(cols, 1, 0, 100, 50, 0, AGGS5)
    total = len(exp["key"])
    got, cnt, status = gpu_window_agg(cols, 1, 0, 100, 50, 0, AGGS5, cap=total // 3)
    assert status == 0 and cnt == total
    # every written row is a correct group
    ek = {(int(w), int(k)): i for i, (w, k) in enumerate(zip(exp["wstart"], exp["key"]))}
    for r in range(len(got["key"])):
        i = ek[(int(got["wstart"][r]), int(got["key"][r]))]
        assert int(got["aggs"][0][r]) == int(exp["aggs"][0][i])


def one_hot_key_cols(lms, n_panes, rows_per_pane, pane_ms, cold_keys=0, seed=0):
    """One key with rows in n_panes consecutive panes (rows_per_pane each),
    plus optional cold keys spread over the same span."""
    rng = np.random.default_rng(seed)
    ts = np.repeat(np.arange(n_panes, dtype=np.int64) * pane_ms, rows_per_pane)
    ts += rng.integers(0, pane_ms, ts.size)
    key = np.full(ts.size, 77, np.int64)
    if cold_keys:
        cts = rng.integers(0, n_panes * pane_ms, cold_keys, dtype=np.int64)
        ts = np.concatenate([ts, cts])
        key = np.concatenate([key, rng.integers(1000, 1000 + cold_keys // 3, cold_keys, dtype=np.int64)])
    perm = rng.permutation(ts.size)
    ts, key = ts[perm], key[perm]
    val = rng.integers(-1000, 1000, ts.size, dtype=np.int32)
    f = rng.standard_normal(ts.size).astype(np.float32)
    return [ts, key, val, f]


@pytest.mark.parametrize("length,slide,rows_per_pane,cold", [
    (1, 0, 1, 0),          # tumbling 1 ms over 10 s: one pane per row, one key
    (1, 0, 3, 5000),       # three rows per pane: a split (pieces + merge) partition
    (50, 10, 1, 3000),     # sliding, window of 5 panes
    (30, 20, 2, 0),        # sliding with slide of 2 panes (window anchors every other pane)
])
def test_window_agg_key_with_more_panes_than_a_table(lms, length, slide, rows_per_pane, cold):
    """A key holding more panes than one workgroup table is aggregated over
    ranges of its windows instead of failing."""
    pane = int(np.gcd(length, slide)) if slide else length
    n_panes = 10000
    log(f"many panes len={length} slide={slide} rows/pane={rows_per_pane} cold={cold}")
    assert n_panes > lms.pane_limit(len(AGGS5))
    cols = one_hot_key_cols(lms, n_panes, rows_per_pane, pane, cold, seed=length + slide)
    got, cnt, status = gpu_window_agg(cols, 1, 0, length, slide, 0, AGGS5)
    assert status == 0
    assert_window_equal(got, oracle.window_agg(cols, 1, 0, length, slide, 0, AGGS5), AGGS5, "many panes")


def test_window_agg_window_spanning_more_panes_than_a_table_reports_capacity(lms):
    limit = lms.pane_limit(len(AGGS5))
    n = 4 * limit
    cols = [np.arange(n, dtype=np.int64), np.zeros(n, np.int64), np.ones(n, np.int32), np.zeros(n, np.float32)]
    # one window of n ms sliding by 1 ms: every window of the key holds up to n non-empty panes
    got, cnt, status = gpu_window_agg(cols, 1, 0, n, 1, 0, AGGS5, cap=1 << 16)
    assert status == lms.LMS_ECAPACITY


def test_window_agg_int32_key_and_ts():
    n = 100000
    rng = np.random.default_rng(8)
    cols = [rng.integers(-100000, 100000, n, dtype=np.int32), rng.integers(0, 900, n, dtype=np.int32),
            rng.integers(0, 100, n, dtype=np.int32), rng.random(n, dtype=np.float32)]
    got, cnt, status = gpu_window_agg(cols, 1, 0, 5000, 2500, 0, AGGS5)
    assert status == 0
    assert_window_equal(got, oracle.window_agg(cols, 1, 0, 5000, 2500, 0, AGGS5), AGGS5, "int32")


def test_window_agg_is_deterministic_on_integers():
    cols = datagen.config1(400000)
    aggs = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2)]
    a, _, _ = gpu_window_agg(cols, 1, 0, 10000, 1000, 0, aggs)
    b, _, _ = gpu_window_agg(cols, 1, 0, 10000, 1000, 0, aggs)
    assert_window_equal(a, b, aggs, "repeat")


# ---------------------------------------------------------------- join

@pytest.mark.parametrize("nb,npr,dup,kdt", [(0, 100, False, np.int64), (1000, 0, False, np.int64),
                                            (1 << 12, 50000, False, np.int64), (5000, 70001, True, np.int64),
                                            (3000, 40000, True, np.int32)])
def test_hash_join_parity(lms, nb, npr, dup, kdt):
    log(f"join nb={nb} np={npr} dup={dup}")
    if dup:
        bk, bp = datagen.static_table_dup(nb, max(1, nb // 2))
    else:
        bk, bp = datagen.static_table(nb)
    pk = datagen.zipf_keys(np.random.default_rng(7), npr, 1.1, max(1, nb))
    if kdt == np.int32:
        bk = (bk & 0x7FFF).astype(np.int32)
        pk = (pk & 0x7FFF).astype(np.int32)
    t = lms.lms_join_build(torch.from_numpy(bk).cuda(), torch.from_numpy(bp).cuda())
    mult = t.max_mult()
    if nb:
        assert mult == int(np.unique(bk, return_counts=True)[1].max())
    idx, pay, d = lms.lms_hash_join(t, torch.from_numpy(pk).cuda())
    torch.cuda.synchronize()
    m, status = [int(x) for x in d.cpu()]
    assert status == 0
    ei, ep = oracle.hash_join(bk, bp, pk)
    assert m == len(ei)
    gi = idx[:m].cpu().numpy().astype(np.uint32).astype(np.int64)
    gp = pay[:m].cpu().numpy()
    np.testing.assert_array_equal(gi, ei)  # grouped by ascending probe row
    o1 = np.lexsort((gp, gi))
    o2 = np.lexsort((ep, ei))
    np.testing.assert_array_equal(gp[o1], ep[o2])
    t.free()


def test_hash_join_capacity_below_count(lms):
    bk, bp = datagen.static_table(1024)
    pk = np.tile(bk, 5)
    t = lms.lms_join_build(torch.from_numpy(bk).cuda(), torch.from_numpy(bp).cuda())
    idx, pay, d = lms.lms_hash_join(t, torch.from_numpy(pk).cuda(), cap=100)
    torch.cuda.synchronize()
    assert int(d[0]) == len(pk)
    ei, ep = oracle.hash_join(bk, bp, pk)
    np.testing.assert_array_equal(idx[:100].cpu().numpy(), ei[:100])
    np.testing.assert_array_equal(pay[:100].cpu().numpy(), ep[:100])

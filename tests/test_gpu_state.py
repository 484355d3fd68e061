"""GPU parity of the device-resident window state: a stream split into
micro-batches, updated batch by batch and emitted as the watermark advances,
must give exactly the oracle's windowed group-by over the whole stream, for
every split (stream-split invariance); late rows and capacity limits are
counted, never silently merged."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import assert_window_equal, log, to_dev
from oracle import AVG, COUNT, LT, MAX, MIN, SUM
from paper_2111_04289_amd import datagen

pytestmark = pytest.mark.gpu

AGGS = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3), (SUM, 4)]
PREDS = [(2, LT, 700)]
PROJS = [(2, 3, -5)]


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def stream_cols(seed, n, nkeys=3000, span=40000, t0=0):
    rng = np.random.default_rng(seed)
    ts = np.sort(rng.integers(t0, t0 + span, n, dtype=np.int64))
    key = datagen.splitmix64(rng.integers(0, nkeys, n).astype(np.uint64)).view(np.int64)
    key[::501] = np.iinfo(np.int64).min  # the dictionary's empty-marker value is an ordinary key
    val = rng.integers(-1000, 1000, n, dtype=np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


def collect(groups, d):
    torch.cuda.synchronize()
    cnt, status = [int(x) for x in d.cpu()]
    assert status == 0, status
    m = min(cnt, groups.cap)
    assert cnt <= groups.cap
    return {"key": groups.key[:m].cpu().numpy(), "wstart": groups.wstart[:m].cpu().numpy(),
            "aggs": [a[:m].cpu().numpy() for a in groups.aggs]}


def concat(parts, nagg):
    return {"key": np.concatenate([p["key"] for p in parts]), "wstart": np.concatenate([p["wstart"] for p in parts]),
            "aggs": [np.concatenate([p["aggs"][k] for p in parts]) for k in range(nagg)]}


def run_stream(lms, cols, cuts, window, ring=512, max_windows=1 << 20):
    st = lms.WindowState(window, AGGS, max_keys=4096, ring_panes=ring)
    dev = to_dev(cols)
    parts = []
    bounds = [0] + list(cuts) + [len(cols[0])]
    for b in range(len(bounds) - 1):
        lo, hi = bounds[b], bounds[b + 1]
        st.update([c[lo:hi] for c in dev], 1, PREDS, PROJS)
        wm = int(cols[0][hi]) if hi < len(cols[0]) else int(cols[0][-1])  # rows with ts < wm have all arrived
        parts.append(collect(*st.emit(wm, cap=1 << 18, max_windows=max_windows)))
    for _ in range(100):  # drain
        g, d = st.emit(flush=True, cap=1 << 18, max_windows=max_windows)
        p = collect(g, d)
        if len(p["key"]) == 0 and st.info()["emit_hi"] < st.info()["emit_lo"]:
            break
        parts.append(p)
    info = st.info()
    st.free()
    return concat(parts, len(AGGS)), info


@pytest.mark.parametrize("length,slide,origin", [(1000, 0, 0), (10000, 1000, 0), (3000, 2000, 7), (700, 300, -50)])
@pytest.mark.parametrize("nbatches", [1, 7, 60])
def test_stream_split_invariance(lms, length, slide, origin, nbatches):
    log(f"wstate window={length}/{slide}/{origin} batches={nbatches}")
    cols = stream_cols(length + slide + nbatches, 60000)
    rng = np.random.default_rng(nbatches)
    cuts = np.sort(rng.choice(np.arange(1, len(cols[0])), nbatches - 1, replace=False)) if nbatches > 1 else []
    w = lms.Window(0, length, slide, origin)
    got, info = run_stream(lms, cols, cuts, w)
    exp = oracle.window_agg(cols, 1, 0, length, slide, origin, AGGS, PREDS, PROJS)
    assert info["late_rows"] == 0 and info["dropped_rows"] == 0 and info["status"] == 0
    assert_window_equal(got, exp, AGGS, f"stream {length}/{slide} in {nbatches} batches")
    # each (key, window) emitted once
    pairs = set(zip(got["key"].tolist(), got["wstart"].tolist()))
    assert len(pairs) == len(got["key"])


def test_emit_in_window_steps(lms):
    """max_windows bounds the windows per call; repeated calls continue in order."""
    cols = stream_cols(5, 20000, span=20000)
    w = lms.Window(0, 4000, 1000, 0)
    got, _ = run_stream(lms, cols, [5000, 15000], w, ring=64, max_windows=1)
    exp = oracle.window_agg(cols, 1, 0, 4000, 1000, 0, AGGS, PREDS, PROJS)
    assert_window_equal(got, exp, AGGS, "one window per emit")


def test_late_rows_are_counted_and_dropped(lms):
    cols = stream_cols(9, 10000, span=20000, t0=0)
    w = lms.Window(0, 2000, 1000, 0)
    st = lms.WindowState(w, AGGS, max_keys=4096, ring_panes=32)
    st.update(to_dev(cols), 1, PREDS, PROJS)
    g, d = st.emit(watermark=12000, cap=1 << 18)
    collect(g, d)
    # windows [s, s + 2000) with s + 2000 <= 12000 are out: s <= 10000, next window 11 -> panes < 11 are late
    old = stream_cols(10, 3000, span=20000, t0=0)
    st.update(to_dev(old), 1, PREDS, PROJS)
    info = st.info()
    passing = old[2] < 700
    assert info["late_rows"] == int((passing & (old[0] < 11000)).sum())
    assert info["status"] == 0 and info["next_window"] == 11
    st.free()


def test_ring_overflow_sets_capacity_status(lms):
    cols = stream_cols(11, 5000, span=100000)
    w = lms.Window(0, 1000, 0, 0)
    st = lms.WindowState(w, [(COUNT, 0)], max_keys=4096, ring_panes=4)  # 100 panes in flight, ring of 4
    st.update(to_dev(cols), 1)
    info = st.info()
    assert info["status"] == lms.LMS_ECAPACITY and info["dropped_rows"] > 0
    st.free()


def test_key_dictionary_full(lms):
    cols = stream_cols(12, 20000, nkeys=5000, span=1000)
    st = lms.WindowState(lms.Window(0, 1000, 0, 0), [(COUNT, 0)], max_keys=100, ring_panes=4)
    st.update(to_dev(cols), 1)
    info = st.info()
    assert info["status"] == lms.LMS_ECAPACITY and info["dropped_rows"] > 0
    st.free()

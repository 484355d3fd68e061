"""Pins of the oracle's Table III query shapes (window_query: composite group
keys, HAVING, ORDER BY an aggregate; window_self_join: LR1's join of the
stream with its own window) against brute-force loops, a library routine and
invariants."""
import numpy as np
import pytest

import brute
import oracle
from oracle import AVG, COUNT, EQ, GE, LT, MAX, MIN, SUM


def small_cols(seed, n, nk=(3, 2, 4), tspan=60):
    rng = np.random.default_rng(seed)
    ts = rng.integers(-tspan // 2, tspan, n).astype(np.int64)
    k1 = rng.integers(0, nk[0], n).astype(np.int32)
    k2 = rng.integers(-1, nk[1] - 1, n).astype(np.int64)
    k3 = rng.integers(0, nk[2], n).astype(np.int32)
    val = rng.integers(-50, 50, n).astype(np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, k1, k2, k3, val, f]


AGGS = [(COUNT, 0), (SUM, 4), (MIN, 4), (MAX, 6), (AVG, 5)]


@pytest.mark.parametrize("seed", range(8))
def test_composite_key_query_matches_brute_force(seed):
    cols = small_cols(seed, 40 + 7 * seed)
    length, slide = [(10, 0), (20, 5), (15, 10), (9, 6)][seed % 4]
    preds = [(4, GE, -30)] if seed % 2 else []
    projs = [(4, 3, 1)]
    key_cols = [1, 2, 3][: 1 + seed % 3]
    got = oracle.window_query(cols, key_cols, 0, length, slide, 0, AGGS, preds, projs)
    exp = brute.window_query([list(c) for c in cols], key_cols, 0, length, slide, 0, AGGS, preds, projs)
    assert len(got["wstart"]) == len(exp)
    for g in range(len(got["wstart"])):
        t = tuple(int(got["keys"][j][g]) for j in range(len(key_cols)))
        want = exp[(int(got["wstart"][g]), t)]
        for k, (fn, _) in enumerate(AGGS):
            if fn == AVG:
                assert abs(got["aggs"][k][g] - want[k]) <= 1e-12 * max(1.0, abs(want[k]))
            else:
                assert int(got["aggs"][k][g]) == int(want[k])
    # sorted by (window start, key tuple)
    order = np.lexsort(tuple(reversed(got["keys"])) + (got["wstart"],))
    assert np.array_equal(order, np.arange(len(order)))


def test_composite_key_equals_single_key_on_tuple_ids():
    """The tuple grouping equals the single-key oracle run on a dense id of
    each distinct tuple (np.unique over rows)."""
    cols = small_cols(11, 5000, nk=(5, 3, 7), tspan=3000)
    tup = np.stack([cols[1].astype(np.int64), cols[2], cols[3].astype(np.int64)], axis=1)
    uniq, ids = np.unique(tup, axis=0, return_inverse=True)
    ids = ids.reshape(-1).astype(np.int64)
    aggs = [(COUNT, 0), (SUM, 4), (MIN, 4), (MAX, 4), (AVG, 5)]
    got = oracle.window_query(cols, [1, 2, 3], 0, 300, 100, 0, aggs)
    single = oracle.window_agg(cols + [ids], 6, 0, 300, 100, 0, aggs)
    assert len(got["wstart"]) == len(single["key"])
    gi = np.lexsort((np.stack(got["keys"]).T @ np.array([1 << 40, 1 << 20, 1]), got["wstart"]))
    sk = uniq[single["key"]]
    si = np.lexsort((sk @ np.array([1 << 40, 1 << 20, 1]), single["wstart"]))
    assert np.array_equal(got["wstart"][gi], single["wstart"][si])
    for j in range(3):
        assert np.array_equal(got["keys"][j][gi], sk[si, j])
    for k in range(len(aggs)):
        assert np.array_equal(got["aggs"][k][gi], single["aggs"][k][si])


def test_having_keeps_exactly_the_satisfying_groups():
    cols = small_cols(3, 3000, tspan=900)
    full = oracle.window_query(cols, [1, 3], 0, 90, 30, 0, AGGS)
    hv = oracle.window_query(cols, [1, 3], 0, 90, 30, 0, AGGS, having=(4, LT, 0.0))
    keep = full["aggs"][4] < 0.0
    assert 0 < keep.sum() < len(keep)
    assert np.array_equal(hv["wstart"], full["wstart"][keep])
    for k in range(len(AGGS)):
        assert np.array_equal(hv["aggs"][k], full["aggs"][k][keep])
    eq = oracle.window_query(cols, [1], 0, 90, 30, 0, AGGS, having=(0, EQ, 3))
    assert (eq["aggs"][0] == 3).all()


@pytest.mark.parametrize("desc", [False, True])
def test_order_by_aggregate_within_each_window(desc):
    cols = small_cols(5, 2000, tspan=600)
    got = oracle.window_query(cols, [1, 2], 0, 60, 20, 0, AGGS, order_by=(1, desc))
    ws, s = got["wstart"], got["aggs"][1]
    assert (np.diff(ws) >= 0).all()
    same = np.diff(ws) == 0
    step = np.diff(s)
    assert ((step <= 0) if desc else (step >= 0))[same].all()
    # the same multiset of groups as the unordered query
    plain = oracle.window_query(cols, [1, 2], 0, 60, 20, 0, AGGS)
    a = np.stack([ws, got["keys"][0], got["keys"][1], s])
    b = np.stack([plain["wstart"], plain["keys"][0], plain["keys"][1], plain["aggs"][1]])
    assert np.array_equal(a[:, np.lexsort(a[::-1])], b[:, np.lexsort(b[::-1])])


@pytest.mark.parametrize("seed", range(6))
def test_self_join_matches_brute_force(seed):
    cols = small_cols(20 + seed, 30 + 5 * seed, nk=(4, 2, 2), tspan=50)
    length, slide = [(10, 0), (20, 5), (12, 8)][seed % 3]
    preds = [(4, LT, 20)] if seed % 2 else []
    w, l, a = oracle.window_self_join(cols, 1, 0, length, slide, 0, preds)
    exp = brute.window_self_join([list(c) for c in cols], 1, 0, length, slide, 0, preds)
    assert list(zip(w.tolist(), l.tolist(), a.tolist())) == sorted(exp)


def test_self_join_counts_are_squares_of_window_counts():
    """Pairs per window = sum over keys of COUNT(key, window)^2, and the pairs
    with l == a are COUNT itself (every row joins with itself)."""
    cols = small_cols(9, 4000, nk=(50, 2, 2), tspan=2000)
    w, l, a = oracle.window_self_join(cols, 1, 0, 300, 100, 0)
    g = oracle.window_agg(cols, 1, 0, 300, 100, 0, [(COUNT, 0)])
    starts, per = np.unique(w, return_counts=True)
    sq = {}
    diag = {}
    for s, c in zip(g["wstart"], g["aggs"][0]):
        sq[int(s)] = sq.get(int(s), 0) + int(c) * int(c)
        diag[int(s)] = diag.get(int(s), 0) + int(c)
    assert dict(zip(starts.tolist(), per.tolist())) == sq
    ds, dc = np.unique(w[l == a], return_counts=True)
    assert dict(zip(ds.tolist(), dc.tolist())) == diag
    assert (cols[1][l] == cols[1][a]).all()

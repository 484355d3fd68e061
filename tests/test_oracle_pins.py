"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle (oracle/lms_oracle.c through oracle/__init__.py)
against brute-force loops (tests/brute.py), independent library routines
(NumPy, pandas) or invariants of the window definition (Table I SlideTime,
Table III range/slide).  None of these re-types the oracle's code.
"""
import numpy as np
import pandas as pd
import pytest

import brute
import oracle
from oracle import AVG, COUNT, EQ, GE, GT, LE, LT, MAX, MIN, NE, SUM


def tiny(seed, n=None, nkeys=None, tspan=None, neg=False, key64=False):
    rng = np.random.default_rng(seed)
    n = n if n is not None else int(rng.integers(0, 160))
    nkeys = nkeys or int(rng.integers(1, 9))
    tspan = tspan or int(rng.integers(1, 60))
    lo = -tspan if neg else 0
    ts = rng.integers(lo, tspan, n, dtype=np.int64)
    if key64:
        key = (rng.integers(0, nkeys, n).astype(np.int64) * np.int64(0x1F2E3D4C5B6A7988)) ^ np.int64(-1234567)
    else:
        key = rng.integers(0, nkeys, n, dtype=np.int32)
    val = rng.integers(-50, 50, n, dtype=np.int32)
    f = rng.standard_normal(n).astype(np.float32)
    return [ts, key, val, f]


def as_lists(cols):
    return [[(float(x) if c.dtype.kind == "f" else int(x)) for x in c] for c in cols]


def oracle_dict(res):
    d = {}
    for g in range(len(res["key"])):
        d[(int(res["wstart"][g]), int(res["key"][g]))] = [a[g] for a in res["aggs"]]
    return d


def assert_groups_equal(got, exp, aggs):
    assert set(got) == set(exp)
    for k in exp:
        for a, (fn, _) in enumerate(aggs):
            if fn == AVG:
                assert got[k][a] == pytest.approx(exp[k][a], rel=1e-12, abs=1e-12), k
            else:
                assert int(got[k][a]) == int(exp[k][a]), (k, a)


AGGS_ALL = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3), (SUM, 4), (AVG, 2)]


@pytest.mark.parametrize("seed", range(40))
def test_window_agg_matches_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    cols = tiny(seed, neg=bool(seed % 3 == 0), key64=bool(seed % 2))
    length = int(rng.integers(1, 12))
    slide = int(rng.integers(0, length + 1))  # 0 = tumbling
    origin = int(rng.integers(-7, 8))
    preds = [(2, int(rng.integers(0, 6)), int(rng.integers(-30, 30)))] if seed % 4 else []
    projs = [(2, int(rng.integers(-3, 4)), int(rng.integers(-5, 6)))]
    got = oracle_dict(oracle.window_agg(cols, 1, 0, length, slide, origin, AGGS_ALL, preds, projs))
    exp = brute.window_agg(as_lists(cols), 1, 0, length, slide, origin, AGGS_ALL, preds, projs,
                           bits=[64, 64 if cols[1].dtype == np.int64 else 32, 32, 32])
    assert_groups_equal(got, exp, AGGS_ALL)


@pytest.mark.parametrize("seed", range(25))
def test_filter_project_matches_brute_force_and_numpy(seed):
    rng = np.random.default_rng(seed)
    cols = tiny(seed, n=int(rng.integers(0, 300)))
    preds = [(2, int(rng.integers(0, 6)), int(rng.integers(-40, 40))),
             (3, int(rng.integers(0, 6)), 0, float(rng.normal()))][: int(rng.integers(0, 3))]
    keep = [0, 1, 3]
    projs = [(2, 2, 0), (0, int(rng.integers(-5, 5)), 7)]
    got = oracle.filter_project(cols, preds, keep, projs)
    exp = brute.filter_project(as_lists(cols), preds, keep, projs, bits=[64, 32, 32, 32])
    for j in range(len(exp)):
        conv = float if got[j].dtype.kind == "f" else int
        assert [conv(x) for x in got[j]] == exp[j]
    # numpy: boolean mask and flatnonzero gather
    mask = np.ones(len(cols[0]), bool)
    ops = [np.less, np.less_equal, np.greater, np.greater_equal, np.equal, np.not_equal]
    for p in preds:
        c = cols[p[0]]
        mask &= ops[p[1]](c, p[3] if c.dtype.kind == "f" else p[2])
    idx = np.flatnonzero(mask)
    assert len(got[0]) == int(mask.sum())
    np.testing.assert_array_equal(got[0], cols[0][idx])
    np.testing.assert_array_equal(got[2], cols[3][idx])
    np.testing.assert_array_equal(got[3], (cols[2][idx].astype(np.int64) * 2).astype(np.int32))


def test_projection_wraps_int32():
    val = np.array([2**30, -2**31, 2**31 - 1, 7], np.int32)
    cols = [np.zeros(4, np.int64), np.zeros(4, np.int32), val, np.zeros(4, np.float32)]
    got = oracle.filter_project(cols, [], [], [(2, 2, 0), (2, 3, 5)])
    np.testing.assert_array_equal(got[0], np.array([-2**31, 0, -2, 14], np.int32))
    np.testing.assert_array_equal(got[1], ((val.astype(np.int64) * 3 + 5) & 0xFFFFFFFF).astype(np.uint32).view(np.int32))


def test_window_sum_of_wrapping_projection():
    # v = val * 5 + 3 wraps modulo 2^32 before it is summed (the projection keeps the int32 width)
    rng = np.random.default_rng(9)
    n = 120
    cols = [rng.integers(0, 40, n, dtype=np.int64), rng.integers(0, 3, n, dtype=np.int32),
            rng.integers(2**29, 2**31 - 1, n, dtype=np.int32), np.zeros(n, np.float32)]
    aggs = [(SUM, 4), (MIN, 4), (MAX, 4)]
    got = oracle_dict(oracle.window_agg(cols, 1, 0, 10, 5, 0, aggs, [], [(2, 5, 3)]))
    exp = brute.window_agg(as_lists(cols), 1, 0, 10, 5, 0, aggs, [], [(2, 5, 3)], bits=[64, 32, 32, 32])
    assert_groups_equal(got, exp, aggs)
    assert any(v[1] < 0 for v in exp.values())  # the wrap is exercised


def test_predicate_nan_semantics():
    f = np.array([np.nan, 1.0, -1.0], np.float32)
    cols = [np.arange(3, dtype=np.int64), np.zeros(3, np.int32), np.zeros(3, np.int32), f]
    for op, expect in [(LT, [2]), (LE, [2]), (GT, [1]), (GE, [1]), (EQ, []), (NE, [0, 1, 2])]:
        got = oracle.filter_project(cols, [(3, op, 0, 0.0)], [0], [])
        assert list(got[0]) == expect, op


def test_tumbling_invariants_config0_shape():
    from paper_2111_04289_amd import datagen
    cols = datagen.config0()
    res = oracle.window_agg(cols, 1, 0, 1000, 0, 0, [(COUNT, 0), (SUM, 4)], [(2, LT, 500)], [(2, 2, 0)])
    mask = cols[2] < 500
    assert res["aggs"][0].sum() == mask.sum()  # sum of per-window counts = filtered rows
    assert res["aggs"][1].sum() == (cols[2][mask].astype(np.int64) * 2).sum()
    assert len(res["key"]) <= 10 * 1024
    # group count close to the occupancy expectation 10240 * (1 - e^-3.2)
    assert abs(len(res["key"]) - 10240 * (1 - np.exp(-mask.sum() / 10240))) < 150


def test_tumbling_single_key_equals_bincount():
    rng = np.random.default_rng(5)
    n = 5000
    ts = rng.integers(0, 10000, n, dtype=np.int64)
    cols = [ts, np.zeros(n, np.int32), rng.integers(0, 1000, n, dtype=np.int32), np.zeros(n, np.float32)]
    res = oracle.window_agg(cols, 1, 0, 700, 0, 0, [(COUNT, 0)])
    bc = np.bincount(ts // 700)
    nz = np.flatnonzero(bc)
    np.testing.assert_array_equal(res["wstart"], nz * 700)
    np.testing.assert_array_equal(res["aggs"][0], bc[nz])


@pytest.mark.parametrize("length,slide", [(1000, 0), (10000, 1000), (3000, 1000), (1000, 400), (7, 3)])
def test_pandas_groupby_cross_check(length, slide):
    cols = tiny(77, n=4000, nkeys=50, tspan=40000, neg=True, key64=True)
    S = slide or length
    res = oracle.window_agg(cols, 1, 0, length, slide, 123, [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2), (AVG, 3)],
                            [(2, GE, -20)])
    df = pd.DataFrame({"ts": cols[0], "key": cols[1], "val": cols[2].astype(np.int64), "f": cols[3].astype(np.float64)})
    df = df[df.val >= -20]
    # expand each row into every window it belongs to (Expand semantics)
    parts = []
    kmax = (df.ts - 123) // S
    for d in range(0, length // S + 2):
        k = kmax - d
        s = 123 + k * S
        sel = s + length > df.ts
        parts.append(df[sel].assign(ws=s[sel]))
    ex = pd.concat(parts)
    g = ex.groupby(["ws", "key"]).agg(cnt=("val", "size"), sm=("val", "sum"), mn=("val", "min"), mx=("val", "max"),
                                      av=("f", "mean")).reset_index()
    assert len(g) == len(res["key"])
    np.testing.assert_array_equal(g.ws.values, res["wstart"])
    np.testing.assert_array_equal(g.key.values, res["key"])
    for j, c in enumerate(["cnt", "sm", "mn", "mx"]):
        np.testing.assert_array_equal(g[c].values, res["aggs"][j])
    np.testing.assert_allclose(g.av.values, res["aggs"][4], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("length,slide", [(10, 1), (10, 5), (12, 4), (9, 9), (30, 10)])
def test_sliding_count_invariant(length, slide):
    # each passing row lies in exactly length/slide windows when slide divides length
    cols = tiny(3, n=3000, nkeys=20, tspan=500, neg=True)
    res = oracle.window_agg(cols, 1, 0, length, slide, -4, [(COUNT, 0), (SUM, 2)], [(2, LT, 10)])
    mask = cols[2] < 10
    assert res["aggs"][0].sum() == (length // slide) * mask.sum()
    assert res["aggs"][1].sum() == (length // slide) * cols[2][mask].astype(np.int64).sum()


@pytest.mark.parametrize("length,slide,origin", [(10, 1, 0), (10, 2, 3), (6, 4, -5), (9, 6, 1)])
def test_sliding_equals_merge_of_tumbling_panes(length, slide, origin):
    # a window of length L sliding by S is the merge of its gcd(L,S)-long tumbling panes
    cols = tiny(11, n=2500, nkeys=12, tspan=200, neg=True, key64=True)
    aggs = [(COUNT, 0), (SUM, 2), (MIN, 2), (MAX, 2)]
    P = int(np.gcd(length, slide))
    slid = oracle_dict(oracle.window_agg(cols, 1, 0, length, slide, origin, aggs))
    panes = oracle_dict(oracle.window_agg(cols, 1, 0, P, 0, origin, aggs))
    merged = {}
    for (ps, key), v in panes.items():
        # windows s = origin + k*slide containing pane [ps, ps + P)
        kmax = (ps - origin) // slide
        k = kmax
        while origin + k * slide + length >= ps + P:
            s = origin + k * slide
            if s <= ps:
                m = merged.setdefault((s, key), [0, 0, None, None])
                m[0] += v[0]
                m[1] += v[1]
                m[2] = v[2] if m[2] is None else min(m[2], v[2])
                m[3] = v[3] if m[3] is None else max(m[3], v[3])
            k -= 1
    assert set(merged) == set(slid)
    for k, v in slid.items():
        assert [int(x) for x in v] == merged[k], k


def test_slide_equal_length_is_tumbling():
    cols = tiny(21, n=2000, nkeys=7, tspan=300, neg=True)
    aggs = [(COUNT, 0), (SUM, 2), (AVG, 3)]
    a = oracle.window_agg(cols, 1, 0, 25, 25, 4, aggs)
    b = oracle.window_agg(cols, 1, 0, 25, 0, 4, aggs)
    for k in ("key", "wstart"):
        np.testing.assert_array_equal(a[k], b[k])
    for x, y in zip(a["aggs"], b["aggs"]):
        np.testing.assert_array_equal(x, y)


def test_window_group_matches_window_agg():
    cols = tiny(8, n=3000, nkeys=30, tspan=1000, neg=True, key64=True)
    aggs = [(COUNT, 0), (SUM, 4), (MIN, 2), (MAX, 2), (AVG, 3)]
    projs = [(2, 2, 1)]
    preds = [(2, LE, 20)]
    res = oracle.window_agg(cols, 1, 0, 100, 20, 7, aggs, preds, projs)
    rng = np.random.default_rng(0)
    for g in rng.choice(len(res["key"]), 40, replace=False):
        cnt, vals = oracle.window_group(cols, 1, 0, 100, 20, 7, aggs, int(res["key"][g]), int(res["wstart"][g]),
                                        preds, projs)
        assert cnt == res["aggs"][0][g]
        for a in range(4):
            assert vals[a] == res["aggs"][a][g]
        assert vals[4] == pytest.approx(res["aggs"][4][g], rel=1e-12)
    # a misaligned window start and an absent key give an empty group
    assert oracle.window_group(cols, 1, 0, 100, 20, 7, aggs, int(res["key"][0]), 8, preds, projs)[0] == 0


def test_sum_wraps_int64():
    n = 4
    big = np.array([2**62, 2**62, 2**62, 5], np.int64)
    cols = [np.zeros(n, np.int64), np.zeros(n, np.int32), big, np.zeros(n, np.float32)]
    res = oracle.window_agg(cols, 1, 0, 10, 0, 0, [(SUM, 2), (MIN, 2), (MAX, 2)])
    assert res["aggs"][0][0] == np.int64(-(2**62) + 5)  # 3 * 2^62 + 5 modulo 2^64
    assert res["aggs"][1][0] == 5 and res["aggs"][2][0] == 2**62


def test_empty_inputs():
    cols = [np.zeros(0, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32)]
    res = oracle.window_agg(cols, 1, 0, 10, 2, 0, [(COUNT, 0)])
    assert len(res["key"]) == 0
    assert all(len(c) == 0 for c in oracle.filter_project(cols, [(2, LT, 0)], [0, 1], [(2, 2, 0)]))
    i, p = oracle.hash_join(np.zeros(0, np.int64), np.zeros(0, np.int32), np.arange(5, dtype=np.int64))
    assert len(i) == 0


@pytest.mark.parametrize("seed", range(20))
def test_join_matches_brute_force(seed):
    rng = np.random.default_rng(seed)
    nb, npb = int(rng.integers(0, 60)), int(rng.integers(0, 80))
    bk = rng.integers(-5, 15, nb).astype(np.int64 if seed % 2 else np.int32)
    bp = rng.integers(-1000, 1000, nb, dtype=np.int32)
    pk = rng.integers(-8, 18, npb).astype(np.int64)
    i, p = oracle.hash_join(bk, bp, pk)
    exp = brute.hash_join([int(x) for x in bk], [int(x) for x in bp], [int(x) for x in pk])
    assert list(zip(i.tolist(), p.tolist())) == exp


def test_join_pandas_merge_and_unique_keys():
    from paper_2111_04289_amd import datagen
    bk, bp = datagen.static_table(1 << 12)
    pk = datagen.zipf_keys(np.random.default_rng(1), 20000, 1.1, 1 << 12)
    i, p = oracle.hash_join(bk, bp, pk)
    assert len(i) == len(pk)  # unique build keys over the same domain: one match per probe row
    m = pd.merge(pd.DataFrame({"i": np.arange(len(pk)), "k": pk}), pd.DataFrame({"k": bk, "p": bp}), on="k")
    m = m.sort_values(["i", "p"])
    np.testing.assert_array_equal(m.i.values, i)
    np.testing.assert_array_equal(m.p.values, p)
    # duplicate build keys: each probe row gets its key's multiplicity
    dk, dp = datagen.static_table_dup(1 << 12, 1 << 12)
    i2, _ = oracle.hash_join(dk, dp, pk)
    ks, cnt = np.unique(dk, return_counts=True)
    mult = dict(zip(ks.tolist(), cnt.tolist()))
    assert len(i2) == sum(mult.get(int(k), 0) for k in pk)

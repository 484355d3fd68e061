"""Brute-force definitions in pure Python, for tiny inputs only.

These pin the C oracle: they are written independently of it (nested loops
over windows, keys and rows; no sorting, no hashing) and compute the same
definitions from the paper's Table I / Table II semantics.
"""
from __future__ import annotations

import math

LT, LE, GT, GE, EQ, NE = 0, 1, 2, 3, 4, 5
COUNT, SUM, MIN, MAX, AVG = 0, 1, 2, 3, 4


def _cmp(v, op, c):
    return [v < c, v <= c, v > c, v >= c, v == c, v != c][op]


def _wrap(v, bits):
    v &= (1 << bits) - 1
    return v - (1 << bits) if v >= 1 << (bits - 1) else v


def row_value(cols, c, i, projs, bits):
    """Value of extended column c (input columns, then projections) at row i."""
    if c < len(cols):
        return cols[c][i]
    src, mul, add = projs[c - len(cols)]
    return _wrap(int(cols[src][i]) * mul + add, bits[src])


def passes(cols, preds, i):
    for p in preds:
        col, op, ival = p[0], p[1], p[2]
        v = cols[col][i]
        c = p[3] if (isinstance(v, float) and len(p) > 3) else ival
        if not _cmp(v, op, c):
            return False
    return True


def filter_project(cols, preds, keep, projs, bits):
    out = [[] for _ in range(len(keep) + len(projs))]
    for i in range(len(cols[0])):
        if not passes(cols, preds, i):
            continue
        for j, c in enumerate(keep):
            out[j].append(cols[c][i])
        for j in range(len(projs)):
            out[len(keep) + j].append(row_value(cols, len(cols) + j, i, projs, bits))
    return out


def window_agg(cols, key_col, ts_col, length, slide, origin, aggs, preds=(), projs=(), bits=None):
    """Dict (wstart, key) -> list of aggregate values, by looping over every
    candidate window start, every key and every row."""
    n = len(cols[0])
    bits = bits or [32] * len(cols)
    S = slide or length
    if n == 0:
        return {}
    tmin, tmax = min(cols[ts_col]), max(cols[ts_col])
    kmin = (tmin - origin - length) // S - 1
    kmax = (tmax - origin) // S + 1
    keys = sorted(set(cols[key_col]))
    res = {}
    for k in range(kmin, kmax + 1):
        s = origin + k * S
        for key in keys:
            rows = [i for i in range(n)
                    if cols[key_col][i] == key and s <= cols[ts_col][i] < s + length and passes(cols, preds, i)]
            if not rows:
                continue
            vals = []
            for fn, c in aggs:
                xs = [row_value(cols, c, i, projs, bits) for i in rows]
                if fn == COUNT:
                    vals.append(len(rows))
                elif fn == SUM:
                    vals.append(_wrap(sum(int(x) for x in xs), 64))
                elif fn == MIN:
                    vals.append(min(xs))
                elif fn == MAX:
                    vals.append(max(xs))
                else:
                    vals.append(math.fsum(float(x) for x in xs) / len(rows))
            res[(s, key)] = vals
    return res


def hash_join(build_keys, build_payload, probe_keys):
    out = []
    for i, k in enumerate(probe_keys):
        for j, bk in enumerate(build_keys):
            if bk == k:
                out.append((i, build_payload[j]))
    return out


def window_query(cols, key_cols, ts_col, length, slide, origin, aggs, preds=(), projs=(), bits=None):
    """Dict (wstart, key tuple) -> aggregate values, by looping over every
    candidate window start, every key tuple and every row."""
    n = len(cols[0])
    bits = bits or [32] * len(cols)
    S = slide or length
    if n == 0:
        return {}
    tmin, tmax = min(cols[ts_col]), max(cols[ts_col])
    kmin = (tmin - origin - length) // S - 1
    kmax = (tmax - origin) // S + 1
    tuples = sorted({tuple(cols[c][i] for c in key_cols) for i in range(n)})
    res = {}
    for k in range(kmin, kmax + 1):
        s = origin + k * S
        for t in tuples:
            rows = [i for i in range(n)
                    if tuple(cols[c][i] for c in key_cols) == t and s <= cols[ts_col][i] < s + length
                    and passes(cols, preds, i)]
            if not rows:
                continue
            vals = []
            for fn, c in aggs:
                xs = [row_value(cols, c, i, projs, bits) for i in rows]
                if fn == COUNT:
                    vals.append(len(rows))
                elif fn == SUM:
                    vals.append(_wrap(sum(int(x) for x in xs), 64))
                elif fn == MIN:
                    vals.append(min(xs))
                elif fn == MAX:
                    vals.append(max(xs))
                else:
                    vals.append(math.fsum(float(x) for x in xs) / len(rows))
            res[(s, t)] = vals
    return res


def window_self_join(cols, key_col, ts_col, length, slide, origin, preds=()):
    """List of (wstart, l, a) by looping over window starts and all row pairs."""
    n = len(cols[0])
    S = slide or length
    if n == 0:
        return []
    tmin, tmax = min(cols[ts_col]), max(cols[ts_col])
    out = []
    for k in range((tmin - origin - length) // S - 1, (tmax - origin) // S + 2):
        s = origin + k * S
        for l in range(n):
            for a in range(n):
                if (cols[key_col][l] == cols[key_col][a] and s <= cols[ts_col][l] < s + length
                        and s <= cols[ts_col][a] < s + length and passes(cols, preds, l) and passes(cols, preds, a)):
                    out.append((s, l, a))
    return out

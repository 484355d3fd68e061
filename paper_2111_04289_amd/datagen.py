"""Seeded synthetic micro-batches.

This module only draws random columns; it computes nothing the operators
compute.  Both the GPU tests and the CPU oracle checks take their inputs from
here, so that the two sides see identical data.

The paper evaluates on Linear Road and Google cluster-monitoring streams
(Table III, Sec. V-A), which are not available here.  The generators below keep
the shapes the paper states (1000-row datasets, Sec. V-A; integer group keys;
range/slide windows of Table III) and fix the distributions the paper leaves
open: key cardinality, Zipf skew and value ranges.

Every column c of configuration k is drawn from
``numpy.random.default_rng(SeedSequence([k, c]))`` (``[k, b, c]`` for batch b
of a multi-batch stream), so any column can be regenerated on its own.
"""
from __future__ import annotations

import math

import numpy as np

MASK64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) on uint64.

    A bijection of the 64-bit integers; used to turn key ranks into keys that
    look arbitrary, so a hash table that hashes keys is not flattered.
    """
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & MASK64
    with np.errstate(over="ignore"):
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & MASK64
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & MASK64
    return z ^ (z >> np.uint64(31))


def _rng(*seed) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence(list(seed)))


def zipf_ranks(rng: np.random.Generator, n: int, s: float, nkeys: int) -> np.ndarray:
    """n ranks in [1, nkeys] with P(rank = k) proportional to k**-s (inverse CDF)."""
    w = np.arange(1, nkeys + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right") + 1
    return np.minimum(r, nkeys).astype(np.int64)


def zipf_keys(rng, n, s=1.1, nkeys=1 << 20) -> np.ndarray:
    return splitmix64(zipf_ranks(rng, n, s, nkeys) - 1).view(np.int64)


# ---------------------------------------------------------------------------
# Column schema shared by the configurations: ts, key, val, f.
TS, KEY, VAL, F = 0, 1, 2, 3

CONFIG0_ROWS = 65536
CONFIG1_ROWS = 1 << 24
CONFIG1_VAL_CUT = 314573  # val < 314573 keeps 0.3 of uniform [0, 2^20)


def config0(n: int = CONFIG0_ROWS):
    """65,536-row micro-batch: ts int64 ms uniform [0, 10000), key int32 uniform
    [0, 1024), val int32 uniform [0, 1000), f float32 uniform [0, 1)."""
    ts = _rng(0, TS).integers(0, 10000, n, dtype=np.int64)
    key = _rng(0, KEY).integers(0, 1024, n, dtype=np.int32)
    val = _rng(0, VAL).integers(0, 1000, n, dtype=np.int32)
    f = _rng(0, F).random(n, dtype=np.float32)
    return [ts, key, val, f]


def config1(n: int = CONFIG1_ROWS, seed: int = 1, span_ms: int = 60000, nkeys: int = 1 << 20):
    """Sliding-window batch: ts int64 uniform over a 60 s span, key int64 =
    SplitMix64 of a Zipf(1.1) rank over 2^20 keys, val int32 uniform [0, 2^20),
    f float32 standard normal."""
    ts = _rng(seed, TS).integers(0, span_ms, n, dtype=np.int64)
    key = zipf_keys(_rng(seed, KEY), n, 1.1, nkeys)
    val = _rng(seed, VAL).integers(0, 1 << 20, n, dtype=np.int32)
    f = _rng(seed, F).standard_normal(n, dtype=np.float32)
    return [ts, key, val, f]


def stream_batch_sizes(nbatches: int = 256, lo: int = 1024, hi: int = 1 << 23, seed: int = 999):
    """Row counts log-uniform in [lo, hi] for the batched uneven stream."""
    u = _rng(2, seed).random(nbatches)
    return np.floor(np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))).astype(np.int64)


def stream_batch(b: int, n: int):
    """Batch b of the uneven stream: the sliding-window schema (config 1)."""
    ts = _rng(2, b, TS).integers(0, 60000, n, dtype=np.int64)
    key = zipf_keys(_rng(2, b, KEY), n, 1.1, 1 << 20)
    val = _rng(2, b, VAL).integers(0, 1 << 20, n, dtype=np.int32)
    f = _rng(2, b, F).standard_normal(n, dtype=np.float32)
    return [ts, key, val, f]


def static_table(nrows: int = 1 << 20, seed: int = 3):
    """Static join side: unique int64 keys (SplitMix64 of a seeded permutation
    of 0..nrows-1, i.e. the same key domain as the Zipf stream keys) and int32
    payload uniform in [0, 2^31 - 1)."""
    perm = _rng(seed, KEY).permutation(nrows).astype(np.uint64)
    keys = splitmix64(perm).view(np.int64)
    payload = _rng(seed, VAL).integers(0, (1 << 31) - 1, nrows, dtype=np.int32)
    return keys, payload


def static_table_dup(nrows: int = 1 << 20, domain: int = 1 << 20, seed: int = 3):
    """Static side with repeated keys: i.i.d. draws from the key domain
    (about Poisson(1) multiplicities)."""
    r = _rng(seed, KEY, 1).integers(0, domain, nrows, dtype=np.int64).astype(np.uint64)
    keys = splitmix64(r).view(np.int64)
    payload = _rng(seed, VAL, 1).integers(0, (1 << 31) - 1, nrows, dtype=np.int32)
    return keys, payload


def poisson_arrivals(rates_rows_per_s=(1e5, 1e6, 5e6, 1e7), step_s=30.0, dataset_rows=1000, seed=4):
    """Arrival times (seconds) of fixed-size datasets under a Poisson process
    whose row rate steps through `rates` every `step_s` seconds."""
    out = []
    t0 = 0.0
    for k, rate in enumerate(rates_rows_per_s):
        lam = rate / dataset_rows  # datasets per second
        rng = _rng(seed, k)
        expected = int(lam * step_s * 1.2) + 16
        gaps = rng.exponential(1.0 / lam, expected)
        t = t0 + np.cumsum(gaps)
        t = t[t < t0 + step_s]
        out.append(t)
        t0 += step_s
    return np.concatenate(out)

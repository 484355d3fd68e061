"""Host-side pieces of the serving loop (no GPU): the Poisson traffic schedule
and the mapping of datasets to pool rows."""
import numpy as np
import pytest
import torch

serve = pytest.importorskip("paper_2111_04289_amd.serve")


def test_traffic_rates_and_order():
    t = serve.Traffic(rates=(1e5, 1e6), step_s=2.0, seed=3)
    a = t.arrivals_ms()
    assert np.all(np.diff(a) >= 0)
    first = a[a < 2000]
    second = a[(a >= 2000) & (a < 4000)]
    assert len(first) + len(second) == len(a)
    # Poisson counts: mean 200 and 2000 datasets, within 5 standard deviations
    assert abs(len(first) - 200) < 5 * np.sqrt(200)
    assert abs(len(second) - 2000) < 5 * np.sqrt(2000)


def test_stream_rows_wrap_the_pool():
    arr = np.arange(10, dtype=np.float64) * 7.5
    d = serve.StreamData(arr, pool_rows=2500, ds_rows=1000)
    assert d.segments(0, 2) == [(0, 0, 2000)]
    assert d.segments(2, 4) == [(0, 2000, 2500), (500, 0, 1500)]
    ts, key, val = d.host_cols(2, 4, (0, 1, 2))
    assert ts.tolist() == [15] * 1000 + [22] * 1000
    np.testing.assert_array_equal(key.numpy(), np.concatenate([d.key.numpy()[2000:], d.key.numpy()[:1500]]))
    np.testing.assert_array_equal(val.numpy()[:500], d.val.numpy()[2000:2500])

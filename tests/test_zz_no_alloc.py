"""The allocation-free filter+project entry point against the workspace one.

lms_filter_project_noalloc keeps its tile counts in the library's fixed
device array; two calls in a row (the second on a smaller batch, so the
array still holds the first call's larger tile table) must each give exactly
what lms_filter_project gives on the same input, and what the oracle gives.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import log, to_dev
from oracle import GE, LT, NE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lms():
    from paper_2111_04289_amd import lms as m
    return m


def make_cols(seed, n):
    rng = np.random.default_rng(seed)
    return [rng.integers(0, 60000, n, dtype=np.int64),
            rng.integers(-(1 << 40), 1 << 40, n, dtype=np.int64),
            rng.integers(0, 1 << 20, n, dtype=np.int32),
            rng.standard_normal(n).astype(np.float32)]


def run_both(lms, cols, preds, keep, projs):
    dev = to_dev(cols)
    n = len(cols[0])
    ref, dref = lms.lms_filter_project(dev, preds, keep, projs)
    out = [torch.full((n,), -3, dtype=dev[c].dtype, device="cuda") for c in keep]
    out += [torch.full((n,), -3, dtype=dev[p[0]].dtype, device="cuda") for p in projs]
    d = torch.full((2,), -9, dtype=torch.int64, device="cuda")
    lms.lms_filter_project_noalloc(dev, out, d, preds, keep, projs)
    torch.cuda.synchronize()
    m, status = [int(x) for x in d.cpu()]
    mref, sref = [int(x) for x in dref.cpu()]
    assert status == 0 and sref == 0
    assert m == mref
    exp = oracle.filter_project(cols, preds, keep, projs)
    assert m == len(exp[0])
    for j in range(len(out)):
        got = out[j][:m].cpu().numpy()
        np.testing.assert_array_equal(got, ref[j][:m].cpu().numpy(), err_msg=f"column {j} vs workspace entry")
        np.testing.assert_array_equal(got, exp[j], err_msg=f"column {j} vs oracle")
    return m


def test_noalloc_matches_workspace_entry_twice(lms):
    preds = [(2, LT, 314573)]
    keep, projs = [0, 1], [(2, 2, 0)]
    big = make_cols(1, 3_000_017)  # 733 wave tiles, ragged tail
    log("noalloc call 1: 3000017 rows")
    m1 = run_both(lms, big, preds, keep, projs)
    small = make_cols(2, 70_001)  # 18 tiles: the array still holds call 1's counts beyond them
    log("noalloc call 2: 70001 rows")
    m2 = run_both(lms, small, [(2, GE, 1000), (3, NE, 0, 0.5)], [3, 2], [(1, -3, 11)])
    assert m1 > m2 > 0


def test_noalloc_empty_and_limit(lms):
    log("noalloc empty batch")
    m = run_both(lms, make_cols(3, 0), [(2, LT, 5)], [0], [])
    assert m == 0
    limit = lms._lib.lms_filter_project_noalloc_max_rows()
    assert limit == 1 << 28
    # a batch above the limit is refused on the host, before anything runs
    col = torch.zeros(1, dtype=torch.int32, device="cuda")
    arr = (lms.lms_col * 1)()
    arr[0].data = col.data_ptr()
    arr[0].dtype = 0
    b = lms.lms_batch(arr, 1, 0, limit + 1)
    o = lms.lms_batch(arr, 1, 0, limit + 1)
    keep = (ctypes.c_int32 * 1)(0)
    d = torch.zeros(2, dtype=torch.int64, device="cuda")
    rc = lms._lib.lms_filter_project_noalloc(ctypes.byref(b), None, 0, keep, 1, None, 0, ctypes.byref(o),
                                             d.data_ptr(), None)
    assert rc == -1
    assert "fixed scratch" in lms.last_error()

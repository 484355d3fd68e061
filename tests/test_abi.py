"""C-ABI checks that need no GPU: the library loads, exports every function
include/lms.h declares, validates arguments on the host, and its host-only
MapDevice planner (Algorithm 2, Eq. 7-9) agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest
import torch

from oracle import plan as oplan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lms.h")

lms = pytest.importorskip("paper_2111_04289_amd.lms")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(lms_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(lms.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lms.ABI_SYMBOLS)


def test_abi_version():
    assert lms._lib.lms_abi_version() == 1


def test_table2_base_costs_match_paper():
    for kind, (_, cost) in oplan.TABLE2.items():
        assert lms.table2_base_cost(kind) == cost
    assert lms.table2_base_cost(99) < 0


@pytest.mark.parametrize("seed", range(30))
def test_plan_matches_oracle(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    kinds = [int(k) for k in rng.integers(0, 8, n)]
    x = float(np.exp(rng.uniform(np.log(0.05), np.log(20))))
    cores = int(rng.integers(1, 25))
    infpt = float(rng.choice([150 * 1024, 64 * 1024, 1e6]))
    bt = float(rng.choice([0.1, 0.05, 0.3]))
    batch = x * infpt * cores
    devs, costs = lms.lms_plan(kinds, batch, cores, infpt, bt)
    odevs, ocosts = oplan.map_device([oplan.TABLE2[k][1] for k in kinds], int(batch), cores, infpt, bt)
    assert devs == odevs
    assert costs == pytest.approx(ocosts, rel=1e-12)


def test_plan_custom_base_costs_and_errors():
    devs, _ = lms.lms_plan([0, 1], 10 * 153600, 1, base_costs=[0.5, 2.0])
    odevs, _ = oplan.map_device([0.5, 2.0], 10 * 153600, 1)
    assert devs == odevs
    with pytest.raises(lms.LmsError):
        lms.lms_plan([0], 1000, 0)
    with pytest.raises(lms.LmsError):
        lms.lms_plan([42], 1000, 1)


def cpu_cols(n=16):
    return [torch.zeros(n, dtype=torch.int64), torch.zeros(n, dtype=torch.int32), torch.zeros(n, dtype=torch.int32),
            torch.zeros(n, dtype=torch.float32)]


@pytest.mark.parametrize("window,aggs,key_col,msg", [
    (lms.Window(0, 10, 11), [(lms.COUNT, 0)], 1, "slide"),
    (lms.Window(0, 0, 0), [(lms.COUNT, 0)], 1, "length"),
    (lms.Window(3, 10, 0), [(lms.COUNT, 0)], 1, "ts column must be integer"),
    (lms.Window(0, 10, 0), [(lms.COUNT, 0)], 3, "key column must be integer"),
    (lms.Window(0, 10, 0), [(lms.SUM, 3)], 1, "integer column"),
    (lms.Window(0, 10, 0), [(lms.MAX, 9)], 1, "out of range"),
    (lms.Window(0, 10, 0), [(7, 2)], 1, "bad function"),
])
def test_window_agg_rejects_bad_arguments(window, aggs, key_col, msg):
    # validation happens on the host before anything is enqueued, so host tensors suffice
    with pytest.raises(lms.LmsError) as e:
        lms.lms_window_agg(cpu_cols(), key_col, window, aggs, cap=4, d_count=torch.zeros(2, dtype=torch.int64),
                           workspace=_HostWs(), stream=0)
    assert e.value.code == lms.LMS_EINVAL
    assert msg in str(e.value)


class _HostWs:
    def get(self, nbytes):
        return torch.zeros(max(nbytes, 1), dtype=torch.uint8)


def test_filter_project_rejects_bad_arguments():
    with pytest.raises(lms.LmsError) as e:
        lms.lms_filter_project(cpu_cols(), [(1, 9, 0)], [0], [], workspace=_HostWs(), stream=0)
    assert e.value.code == lms.LMS_EINVAL
    with pytest.raises(lms.LmsError):
        lms.lms_filter_project(cpu_cols(), [], [0], [(3, 2, 0)], workspace=_HostWs(), stream=0)  # float projection source


def test_workspace_queries_are_positive_and_grow():
    a = lms._lib.lms_filter_project_workspace(1000)
    b = lms._lib.lms_filter_project_workspace(10_000_000)
    assert 0 < a < b
    assert lms._lib.lms_hash_join_workspace(5) > 0
    small = lms.lms_window_agg_workspace(cpu_cols(16), 1, lms.Window(0, 10, 2), [(lms.COUNT, 0), (lms.SUM, 2)])
    assert small > 0
    assert lms.pane_limit(4) >= 1024


@pytest.mark.parametrize("keys,having,order,msg", [
    ([], None, None, "nkey"),
    ([(1, 0, 9)] * 5, None, None, "nkey"),
    ([(1, 0, 1 << 40), (2, 0, 1 << 30)], None, None, "2^62"),
    ([(1, 5, 4), (2, 0, 1)], None, None, "hi < lo"),
    ([(3, 0, 9), (2, 0, 1)], None, None, "integer column"),
    ([(1, 0, 9), (2, 0, 1)], (3, 0, 1), None, "HAVING"),
    ([(1, 0, 9), (2, 0, 1)], None, (2, True), "ORDER BY"),
])
def test_window_query_rejects_bad_arguments(keys, having, order, msg):
    with pytest.raises(lms.LmsError) as e:
        lms.lms_window_query(cpu_cols(), keys, lms.Window(0, 10, 0), [(lms.COUNT, 0), (lms.SUM, 2)], having=having,
                             order=order, cap=4, d_count=torch.zeros(2, dtype=torch.int64), workspace=_HostWs(),
                             stream=0)
    assert e.value.code == lms.LMS_EINVAL
    assert msg in str(e.value)


def test_window_self_join_rejects_bad_arguments():
    with pytest.raises(lms.LmsError) as e:
        lms.lms_window_self_join(cpu_cols(), 3, lms.Window(0, 10, 0), cap=4, d_count=torch.zeros(2, dtype=torch.int64),
                                 workspace=_HostWs(), stream=0)
    assert "key column" in str(e.value)
    with pytest.raises(lms.LmsError):
        lms.lms_window_self_join(cpu_cols(), 1, lms.Window(0, 10, 20), cap=4,
                                 d_count=torch.zeros(2, dtype=torch.int64), workspace=_HostWs(), stream=0)
    assert lms._lib.lms_window_self_join_workspace(1000) > 0

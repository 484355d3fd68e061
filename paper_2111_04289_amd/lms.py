"""ctypes binding of liblms.so (include/lms.h).

Argument marshalling only: every step of the operators runs in the library's
HIP kernels.  torch tensors supply device memory and streams.  Importing this
module loads the library and raises ImportError if it has not been built
(``python -m paper_2111_04289_amd.build``); there is no fallback path.

The functions named like the C entry points (``lms_filter_project``,
``lms_window_agg``, ``lms_join_build``, ``lms_hash_join``, ``lms_plan``) take
torch tensors and plain Python values; they enqueue work on the current (or
given) stream and return device tensors without synchronising.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LMS_LIB_PATH selects another build of the same ABI (e.g. an instrumented one)
LIB_PATH = os.environ.get("LMS_LIB_PATH") or os.path.join(_HERE, "liblms.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_04289_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (lms.h) ------------------------------------------------------
LMS_OK, LMS_EINVAL, LMS_EHIP, LMS_ENOMEM, LMS_ECAPACITY, LMS_ERANGE = 0, -1, -2, -3, -4, -5
I32, I64, F32, F64 = 0, 1, 2, 3
LT, LE, GT, GE, EQ, NE = 0, 1, 2, 3, 4, 5
COUNT, SUM, MIN, MAX, AVG = 0, 1, 2, 3, 4
OP_AGG, OP_FILTER, OP_SHUFFLE, OP_PROJECT, OP_JOIN, OP_EXPAND, OP_SCAN, OP_SORT = range(8)
DEV_CPU, DEV_GPU = 0, 1
PLAN_ANALYTIC, PLAN_LEARNED = 0, 1

_TORCH_DT = {torch.int32: I32, torch.int64: I64, torch.float32: F32, torch.float64: F64}
_DT_TORCH = {v: k for k, v in _TORCH_DT.items()}


class LmsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lms error {code}: {msg}")
        self.code = code


# ---- ABI structs ---------------------------------------------------------------
class lms_col(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lms_batch(ctypes.Structure):
    _fields_ = [("cols", ctypes.POINTER(lms_col)), ("ncols", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("nrows", ctypes.c_int64)]


class lms_pred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("op", ctypes.c_int32), ("ival", ctypes.c_int64), ("fval", ctypes.c_double)]


class lms_proj(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int32), ("reserved", ctypes.c_int32), ("mul", ctypes.c_int64),
                ("add", ctypes.c_int64)]


class lms_window(ctypes.Structure):
    _fields_ = [("ts_col", ctypes.c_int32), ("reserved", ctypes.c_int32), ("len", ctypes.c_int64),
                ("slide", ctypes.c_int64), ("origin", ctypes.c_int64)]


class lms_agg(ctypes.Structure):
    _fields_ = [("fn", ctypes.c_int32), ("col", ctypes.c_int32)]


class lms_groups(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("wstart", ctypes.c_void_p), ("aggs", ctypes.POINTER(ctypes.c_void_p)),
                ("cap", ctypes.c_int64)]


class lms_op_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("ncols", ctypes.c_int32), ("base_cost", ctypes.c_double),
                ("window_s", ctypes.c_double), ("slide_s", ctypes.c_double)]


class lms_batch_stats(ctypes.Structure):
    _fields_ = [("batch_bytes", ctypes.c_int64), ("num_cores", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("selectivity", ctypes.c_double), ("distinct_keys", ctypes.c_int64),
                ("interval_s", ctypes.c_double)]


class lms_cost_params(ctypes.Structure):
    _fields_ = [("infpt_bytes", ctypes.c_double), ("base_trans", ctypes.c_double), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("model", ctypes.c_void_p)]


class lms_trace_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double)]


class lms_multi_config(ctypes.Structure):
    _fields_ = [("nbatch", ctypes.c_int32), ("ma", ctypes.c_int32), ("max_nparts", ctypes.c_int32),
                ("grid_scan", ctypes.c_int32), ("grid_agg", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("agg_lds", ctypes.c_uint64)]


class lms_admit_params(ctypes.Structure):
    _fields_ = [("slide_ms", ctypes.c_double), ("deadline_ms", ctypes.c_double), ("poll_ms", ctypes.c_double),
                ("poll_idle", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lms_admit_decision(ctypes.Structure):
    _fields_ = [("admit", ctypes.c_int32), ("reserved", ctypes.c_int32), ("datasets", ctypes.c_int64),
                ("rows", ctypes.c_int64), ("oldest_arrival_ms", ctypes.c_double), ("est_maxlat_ms", ctypes.c_double),
                ("buffered_datasets", ctypes.c_int64), ("buffered_rows", ctypes.c_int64)]


class lms_admit_stats(ctypes.Structure):
    _fields_ = [("batches_done", ctypes.c_int64), ("admitted", ctypes.c_int64), ("rows_done", ctypes.c_int64),
                ("buffered_rows", ctypes.c_int64), ("avg_thput_rows_per_ms", ctypes.c_double),
                ("mean_maxlat_ms", ctypes.c_double)]


class lms_keypart(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("reserved", ctypes.c_int32), ("lo", ctypes.c_int64), ("hi", ctypes.c_int64)]


class lms_having(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_int32), ("op", ctypes.c_int32), ("ival", ctypes.c_int64), ("fval", ctypes.c_double)]


class lms_order(ctypes.Structure):
    _fields_ = [("agg", ctypes.c_int32), ("descending", ctypes.c_int32)]


class lms_qgroups(ctypes.Structure):
    _fields_ = [("keys", ctypes.POINTER(ctypes.c_void_p)), ("wstart", ctypes.c_void_p),
                ("aggs", ctypes.POINTER(ctypes.c_void_p)), ("cap", ctypes.c_int64)]


class lms_tuning(ctypes.Structure):
    _fields_ = [("chunk_rows", ctypes.c_int32), ("part_rows", ctypes.c_int32), ("piece_rows", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("lds_groups", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_P = ctypes.POINTER
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_SIGS = {
    "lms_abi_version": (ctypes.c_int, []),
    "lms_last_error": (ctypes.c_char_p, []),
    "lms_filter_project_workspace": (_sz, [_i64]),
    "lms_filter_project": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _P(ctypes.c_int32), _i32, _P(lms_proj),
                                          _i32, _P(lms_batch), _vp, _vp, _sz, _vp]),
    "lms_filter_project_noalloc_max_rows": (_i64, []),
    "lms_filter_project_noalloc": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _P(ctypes.c_int32), _i32,
                                                  _P(lms_proj), _i32, _P(lms_batch), _vp, _vp]),
    "lms_window_agg_workspace": (_sz, [_P(lms_batch), _i32, _P(lms_window), _P(lms_agg), _i32]),
    "lms_window_agg_pane_limit": (_i64, [_i32]),
    "lms_window_agg": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _P(lms_proj), _i32, _i32, _P(lms_window),
                                      _P(lms_agg), _i32, _P(lms_groups), _vp, _vp, _sz, _vp]),
    "lms_window_agg_emit": (ctypes.c_int, [_P(lms_groups), _i32, _vp, _vp, _sz, _vp]),
    "lms_window_query_workspace": (_sz, [_P(lms_batch), _P(lms_keypart), _i32, _P(lms_window), _P(lms_agg), _i32,
                                         _i32, _i64]),
    "lms_window_query": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _P(lms_proj), _i32, _P(lms_keypart), _i32,
                                        _P(lms_window), _P(lms_agg), _i32, _P(lms_having), _P(lms_order),
                                        _P(lms_qgroups), _vp, _vp, _sz, _vp]),
    "lms_window_self_join_workspace": (_sz, [_i64]),
    "lms_window_self_join": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _i32, _P(lms_window), _vp, _vp, _vp,
                                            _i64, _vp, _vp, _sz, _vp]),
    "lms_window_agg_multi_workspace": (_sz, [_P(lms_batch), _i32, _i32, _P(lms_window), _P(lms_agg), _i32]),
    "lms_window_agg_multi_prepare": (ctypes.c_int, [_P(lms_batch), _i32, _P(lms_pred), _i32, _P(lms_proj), _i32, _i32,
                                                    _P(lms_window), _P(lms_agg), _i32, _P(lms_groups), _vp, _vp, _sz,
                                                    _P(lms_multi_config), _vp]),
    "lms_window_agg_multi_launch": (ctypes.c_int, [_P(lms_multi_config), _vp, _vp]),
    "lms_wstate_bytes": (_sz, [_i64, _i32, _i32]),
    "lms_wstate_create": (ctypes.c_int, [_P(lms_window), _P(lms_agg), _i32, _i64, _i32, _P(_vp), _vp]),
    "lms_wstate_update": (ctypes.c_int, [_vp, _P(lms_batch), _P(lms_pred), _i32, _P(lms_proj), _i32, _i32, _vp]),
    "lms_wstate_emit": (ctypes.c_int, [_vp, _i64, _i32, _i32, _P(lms_groups), _vp, _vp]),
    "lms_wstate_info": (ctypes.c_int, [_vp, _vp, _vp]),
    "lms_wstate_free": (None, [_vp]),
    "lms_admit_create": (ctypes.c_int, [_P(lms_admit_params), _P(_vp)]),
    "lms_admit_poll": (ctypes.c_int, [_vp, ctypes.c_double, _i64, _vp, _vp, _P(lms_admit_decision)]),
    "lms_admit_done": (ctypes.c_int, [_vp, _i64, ctypes.c_double, ctypes.c_double]),
    "lms_admit_get_stats": (ctypes.c_int, [_vp, _P(lms_admit_stats)]),
    "lms_admit_set_model": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, ctypes.c_double]),
    "lms_admit_predict_ms": (ctypes.c_double, [_vp, _i64]),
    "lms_admit_free": (None, [_vp]),
    "lms_set_tuning": (ctypes.c_int, [_P(lms_tuning)]),
    "lms_get_tuning": (ctypes.c_int, [_P(lms_tuning)]),
    "lms_join_build": (ctypes.c_int, [_P(lms_batch), _i32, _i32, _P(_vp), _vp]),
    "lms_join_max_mult": (_i64, [_vp]),
    "lms_join_build_rows": (_i64, [_vp]),
    "lms_join_free": (None, [_vp]),
    "lms_hash_join_workspace": (_sz, [_i64]),
    "lms_hash_join": (ctypes.c_int, [_vp, _P(lms_batch), _i32, _vp, _vp, _i64, _vp, _vp, _sz, _vp]),
    "lms_cpu_filter_project": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _P(ctypes.c_int32), _i32,
                                              _P(lms_proj), _i32, _P(lms_batch), _P(ctypes.c_int64), _i32]),
    "lms_cpu_window_agg": (ctypes.c_int, [_P(lms_batch), _P(lms_pred), _i32, _P(lms_proj), _i32, _i32,
                                          _P(lms_window), _P(lms_agg), _i32, _P(lms_groups), _P(ctypes.c_int64), _i32]),
    "lms_cpu_hash_join": (ctypes.c_int, [_P(lms_batch), _i32, _i32, _P(lms_batch), _i32, _vp, _vp, _i64,
                                         _P(ctypes.c_int64), _i32]),
    "lms_mlp_create": (ctypes.c_int, [ctypes.c_uint64, _P(_vp)]),
    "lms_mlp_free": (None, [_vp]),
    "lms_mlp_set_params": (ctypes.c_int, [_vp, _vp]),
    "lms_mlp_get_params": (ctypes.c_int, [_vp, _vp]),
    "lms_mlp_workspace": (_sz, [_i64]),
    "lms_mlp_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp]),
    "lms_mlp_adam_step": (ctypes.c_int, [_vp, _vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                         _vp]),
    "lms_mlp_forward": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i32, _vp]),
    "lms_mlp_host_forward": (None, [_vp, _vp, _vp]),
    "lms_mlp_features": (None, [_P(lms_op_desc), _P(lms_batch_stats), _i32, _vp]),
    "lms_bf16_round": (ctypes.c_float, [ctypes.c_float]),
    "lms_trace_enable": (ctypes.c_int, [_i32]),
    "lms_trace_read": (ctypes.c_int, [_P(lms_trace_stat), _i32]),
    "lms_table2_base_cost": (ctypes.c_double, [_i32]),
    "lms_infpt_create": (ctypes.c_int, [ctypes.c_double, _i32, ctypes.c_double, ctypes.c_uint64, _P(_vp)]),
    "lms_infpt_record": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lms_infpt_next": (ctypes.c_double, [_vp, ctypes.c_double]),
    "lms_infpt_free": (None, [_vp]),
    "lms_plan": (ctypes.c_int, [_P(lms_op_desc), _i32, _P(lms_batch_stats), _P(lms_cost_params), _P(ctypes.c_int32),
                                _P(ctypes.c_double)]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

ABI_SYMBOLS = tuple(_SIGS)


def last_error() -> str:
    return (_lib.lms_last_error() or b"").decode()


def _check(rc: int):
    if rc != LMS_OK:
        raise LmsError(rc, last_error())


def _stream_handle(stream) -> int:
    if isinstance(stream, int):  # a raw hipStream_t handle
        return stream
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class _Batch:
    """Keeps the ctypes column array alive alongside the lms_batch."""

    def __init__(self, cols: Sequence[torch.Tensor], nrows: int | None = None):
        self.tensors = list(cols)
        n = {int(t.shape[0]) for t in self.tensors}
        if nrows is None:
            if len(n) > 1:
                raise ValueError("columns differ in length")
            nrows = n.pop() if n else 0
        for t in self.tensors:
            if t.dim() != 1 or not t.is_contiguous() or t.dtype not in _TORCH_DT:
                raise ValueError("columns must be contiguous 1-D int32/int64/float32/float64 tensors")
        self.arr = (lms_col * max(1, len(self.tensors)))()
        for i, t in enumerate(self.tensors):
            self.arr[i].data = t.data_ptr()
            self.arr[i].dtype = _TORCH_DT[t.dtype]
        self.batch = lms_batch(self.arr, len(self.tensors), 0, nrows)


def _preds(preds):
    preds = list(preds)
    arr = (lms_pred * max(1, len(preds)))()
    for i, p in enumerate(preds):
        col, op, ival = p[0], p[1], p[2]
        fval = p[3] if len(p) > 3 else float(ival)
        arr[i] = lms_pred(col, op, int(ival), float(fval))
    return arr, len(preds)


def _projs(projs):
    projs = list(projs)
    arr = (lms_proj * max(1, len(projs)))()
    for i, (src, mul, add) in enumerate(projs):
        arr[i] = lms_proj(src, 0, int(mul), int(add))
    return arr, len(projs)


class Workspace:
    """A grow-only device scratch buffer for the operators.

    Calls that may overlap in time need workspaces of their own (lms.h).
    """

    def __init__(self, device=None):
        self.device = device or torch.device("cuda")
        self.buf = torch.empty(0, dtype=torch.uint8, device=self.device)

    def get(self, nbytes: int) -> torch.Tensor:
        if self.buf.numel() < nbytes:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf


# one default workspace per (device, stream): calls on one stream never
# overlap, calls on different streams never share one
_default_ws: dict = {}


def _torch_stream(stream, device):
    if stream is None:
        return torch.cuda.current_stream(device)
    if isinstance(stream, int):
        return torch.cuda.ExternalStream(stream, device=device)
    return stream


def _ws(workspace, nbytes, device, stream=None):
    device = torch.device(device)
    s = _torch_stream(stream, device) if device.type == "cuda" else None
    if workspace is None:
        key = (str(device), s.cuda_stream if s is not None else stream)
        workspace = _default_ws.setdefault(key, Workspace(device))
    buf = workspace if isinstance(workspace, torch.Tensor) else workspace.get(nbytes)
    if isinstance(workspace, torch.Tensor) and buf.numel() < nbytes:
        raise ValueError(f"workspace of {buf.numel()} bytes is smaller than the {nbytes} needed")
    if s is not None and s.cuda_stream != torch.cuda.current_stream(device).cuda_stream:
        # the buffer is used on another stream than the one it was allocated
        # on: the allocator must not hand it out again before that work ends
        buf.record_stream(s)
    return buf


# ---- filter + project -------------------------------------------------------------

def lms_filter_project(cols, preds=(), keep=(), projs=(), out=None, d_count=None, workspace=None, stream=None):
    """Enqueues filter+project; returns (out_cols, d_count) with out_cols sized n."""
    b = _Batch(cols)
    n = b.batch.nrows
    dev = cols[0].device if cols else torch.device("cuda")
    keep = list(keep)
    projs = list(projs)
    if out is None:
        out = [torch.empty(n, dtype=cols[c].dtype, device=dev) for c in keep]
        out += [torch.empty(n, dtype=cols[p[0]].dtype, device=dev) for p in projs]
    ob = _Batch(out, nrows=n)
    pa, npred = _preds(preds)
    pr, nproj = _projs(projs)
    ka = (ctypes.c_int32 * max(1, len(keep)))(*keep)
    if d_count is None:
        d_count = torch.zeros(2, dtype=torch.int64, device=dev)
    need = _lib.lms_filter_project_workspace(n)
    ws = _ws(workspace, need, dev, stream)
    rc = _lib.lms_filter_project(ctypes.byref(b.batch), pa, npred, ka, len(keep), pr, nproj, ctypes.byref(ob.batch),
                                 d_count.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _check(rc)
    return out, d_count


def lms_filter_project_noalloc(cols, out, d_count, preds=(), keep=(), projs=(), stream=None):
    """Enqueues filter+project with the library's fixed scratch (no workspace).

    The caller supplies the output columns (room for every input row) and the
    device int64[2] count; calls that overlap on one GPU race (lms.h)."""
    b = _Batch(cols)
    keep = list(keep)
    projs = list(projs)
    ob = _Batch(out, nrows=b.batch.nrows)
    pa, npred = _preds(preds)
    pr, nproj = _projs(projs)
    ka = (ctypes.c_int32 * max(1, len(keep)))(*keep)
    rc = _lib.lms_filter_project_noalloc(ctypes.byref(b.batch), pa, npred, ka, len(keep), pr, nproj,
                                         ctypes.byref(ob.batch), d_count.data_ptr(), _stream_handle(stream))
    _check(rc)
    return out, d_count


# ---- windowed group-by ---------------------------------------------------------------

@dataclass
class Window:
    ts_col: int
    length: int
    slide: int = 0
    origin: int = 0

    def c(self):
        return lms_window(self.ts_col, 0, self.length, self.slide, self.origin)


def lms_window_agg_workspace(cols, key_col, window: Window, aggs) -> int:
    b = _Batch(cols)
    aa = (lms_agg * max(1, len(aggs)))(*[lms_agg(f, c) for f, c in aggs])
    w = window.c()
    return int(_lib.lms_window_agg_workspace(ctypes.byref(b.batch), key_col, ctypes.byref(w), aa, len(aggs)))


def pane_limit(nagg: int) -> int:
    return int(_lib.lms_window_agg_pane_limit(nagg))


class Groups:
    """Device output columns of lms_window_agg."""

    def __init__(self, cap: int, aggs, device):
        self.cap = cap
        self.key = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
        self.wstart = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
        self.aggs = [torch.empty(max(cap, 1), dtype=torch.float64 if f == AVG else torch.int64, device=device)
                     for f, _ in aggs]
        self._ptrs = (ctypes.c_void_p * max(1, len(self.aggs)))(*[t.data_ptr() for t in self.aggs])
        self.c = lms_groups(self.key.data_ptr(), self.wstart.data_ptr(), self._ptrs, cap)


def lms_window_agg(cols, key_col, window: Window, aggs, preds=(), projs=(), groups: Groups | None = None,
                   cap: int | None = None, d_count=None, workspace=None, stream=None):
    """Enqueues the windowed group-by; returns (groups, d_count)."""
    b = _Batch(cols)
    n = b.batch.nrows
    dev = cols[0].device
    aggs = list(aggs)
    if groups is None:
        if cap is None:
            slide = window.slide or window.length
            cap = n * (-(-window.length // slide))  # provable bound: each row is in ceil(len/slide) windows
        groups = Groups(cap, aggs, dev)
    if d_count is None:
        d_count = torch.zeros(2, dtype=torch.int64, device=dev)
    pa, npred = _preds(preds)
    pr, nproj = _projs(projs)
    aa = (lms_agg * max(1, len(aggs)))(*[lms_agg(f, c) for f, c in aggs])
    w = window.c()
    need = _lib.lms_window_agg_workspace(ctypes.byref(b.batch), key_col, ctypes.byref(w), aa, len(aggs))
    ws = _ws(workspace, need, dev, stream)
    rc = _lib.lms_window_agg(ctypes.byref(b.batch), pa, npred, pr, nproj, key_col, ctypes.byref(w), aa, len(aggs),
                             ctypes.byref(groups.c), d_count.data_ptr(), ws.data_ptr(), ws.numel(),
                             _stream_handle(stream))
    _check(rc)
    return groups, d_count


class QueryGroups:
    """Device output columns of lms_window_query: one int64 column per key part."""

    def __init__(self, cap: int, nkey: int, aggs, device):
        self.cap = cap
        self.keys = [torch.empty(max(cap, 1), dtype=torch.int64, device=device) for _ in range(nkey)]
        self.wstart = torch.empty(max(cap, 1), dtype=torch.int64, device=device)
        self.aggs = [torch.empty(max(cap, 1), dtype=torch.float64 if f == AVG else torch.int64, device=device)
                     for f, _ in aggs]
        self._kp = (ctypes.c_void_p * max(1, nkey))(*[t.data_ptr() for t in self.keys])
        self._ap = (ctypes.c_void_p * max(1, len(self.aggs)))(*[t.data_ptr() for t in self.aggs])
        self.c = lms_qgroups(self._kp, self.wstart.data_ptr(), self._ap, cap)


def lms_window_query(cols, keys, window: Window, aggs, preds=(), projs=(), having=None, order=None, cap=None,
                     groups: QueryGroups | None = None, d_count=None, workspace=None, stream=None):
    """Enqueues a windowed query with a composite key, HAVING and ORDER BY.

    keys: [(col, lo, hi)] (lo/hi: the column's value domain; ignored for one
    key); having: (agg index, op, value); order: (agg index, descending).
    Returns (groups, d_count)."""
    b = _Batch(cols)
    n = b.batch.nrows
    dev = cols[0].device
    aggs = list(aggs)
    keys = [tuple(k) if len(k) == 3 else (k[0], 0, 0) for k in keys]
    if groups is None:
        if cap is None:
            slide = window.slide or window.length
            cap = n * (-(-window.length // slide))
        groups = QueryGroups(cap, len(keys), aggs, dev)
    if d_count is None:
        d_count = torch.zeros(2, dtype=torch.int64, device=dev)
    pa, npred = _preds(preds)
    pr, nproj = _projs(projs)
    aa = (lms_agg * max(1, len(aggs)))(*[lms_agg(f, c) for f, c in aggs])
    ka = (lms_keypart * max(1, len(keys)))(*[lms_keypart(int(c), 0, int(lo), int(hi)) for c, lo, hi in keys])
    w = window.c()
    hv = None
    if having is not None:
        k, op, v = having
        hv = lms_having(int(k), int(op), 0 if isinstance(v, float) else int(v), float(v))
    od = lms_order(int(order[0]), 1 if order[1] else 0) if order is not None else None
    need = _lib.lms_window_query_workspace(ctypes.byref(b.batch), ka, len(keys), ctypes.byref(w), aa, len(aggs),
                                           1 if order is not None else 0, groups.cap)
    ws = _ws(workspace, need, dev, stream)
    rc = _lib.lms_window_query(ctypes.byref(b.batch), pa, npred, pr, nproj, ka, len(keys), ctypes.byref(w), aa,
                               len(aggs), ctypes.byref(hv) if hv is not None else None,
                               ctypes.byref(od) if od is not None else None, ctypes.byref(groups.c),
                               d_count.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _check(rc)
    return groups, d_count


def lms_window_self_join(cols, key_col, window: Window, preds=(), cap=None, out=None, d_count=None, workspace=None,
                         stream=None):
    """Enqueues the windowed self-join; returns ((wstart, l, a), d_count)."""
    b = _Batch(cols)
    n = b.batch.nrows
    dev = cols[0].device
    if out is None:
        cap = max(1, n) if cap is None else cap
        out = (torch.empty(cap, dtype=torch.int64, device=dev), torch.empty(cap, dtype=torch.int32, device=dev),
               torch.empty(cap, dtype=torch.int32, device=dev))
    cap = out[0].numel() if cap is None else cap
    if d_count is None:
        d_count = torch.zeros(2, dtype=torch.int64, device=dev)
    pa, npred = _preds(preds)
    w = window.c()
    need = _lib.lms_window_self_join_workspace(n)
    ws = _ws(workspace, need, dev, stream)
    rc = _lib.lms_window_self_join(ctypes.byref(b.batch), pa, npred, key_col, ctypes.byref(w), out[0].data_ptr(),
                                   out[1].data_ptr(), out[2].data_ptr(), cap, d_count.data_ptr(), ws.data_ptr(),
                                   ws.numel(), _stream_handle(stream))
    _check(rc)
    return out, d_count


def lms_window_agg_emit(aggs, workspace, groups: Groups | None = None, cap: int | None = None, d_count=None,
                        stream=None):
    """Enqueues the re-emission of the groups of the last lms_window_agg call
    that used ``workspace`` (a Workspace or the tensor it handed out); returns
    (groups, d_count).  The input columns are not read."""
    buf = workspace.buf if isinstance(workspace, Workspace) else workspace
    dev = buf.device
    aggs = list(aggs)
    if groups is None:
        if cap is None:
            raise ValueError("give groups or cap")
        groups = Groups(cap, aggs, dev)
    if d_count is None:
        d_count = torch.zeros(2, dtype=torch.int64, device=dev)
    rc = _lib.lms_window_agg_emit(ctypes.byref(groups.c), len(aggs), d_count.data_ptr(), buf.data_ptr(), buf.numel(),
                                  _stream_handle(stream))
    _check(rc)
    return groups, d_count


class MultiJob:
    """The windowed group-by of many micro-batches, one persistent launch per stage.

    ``prepare`` writes the batches' descriptors into the job's workspace (and
    may be called again with other batches of the same schema); ``launch``
    enqueues the kernels, which read only the workspace, so it can be captured
    in a graph once and replayed after each ``prepare``.  Batch b's result is in
    ``groups[b]`` and ``d_counts[b]`` ([count, status]).
    """

    def __init__(self, key_col, window: Window, aggs, preds=(), projs=(), device=None):
        self.key_col, self.window, self.aggs = key_col, window, list(aggs)
        self.preds, self.projs = list(preds), list(projs)
        self.device = device or torch.device("cuda")
        self.ws = torch.empty(0, dtype=torch.uint8, device=self.device)
        self.cfg = lms_multi_config()
        self.launch_cfg = None  # the limits launches are configured for
        self._keep = None

    def _arrays(self, batches):
        bs = [_Batch(c) for c in batches]
        arr = (lms_batch * len(bs))(*[b.batch for b in bs])
        aa = (lms_agg * max(1, len(self.aggs)))(*[lms_agg(f, c) for f, c in self.aggs])
        return bs, arr, aa

    def workspace_bytes(self, batches) -> int:
        bs, arr, aa = self._arrays(batches)
        w = self.window.c()
        need = int(_lib.lms_window_agg_multi_workspace(arr, len(bs), self.key_col, ctypes.byref(w), aa,
                                                       len(self.aggs)))
        if need == 0:
            raise LmsError(LMS_EINVAL, last_error() or "invalid multi-batch job")
        return need

    def reserve(self, nbytes: int):
        """Allocates the workspace up front (it cannot move once launches are frozen)."""
        if self.launch_cfg is not None and nbytes > self.ws.numel():
            raise LmsError(LMS_ENOMEM, "the workspace of a frozen job cannot grow")
        if self.ws.numel() < nbytes:
            self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def prepare(self, batches, groups=None, caps=None, d_counts=None, stream=None):
        bs, arr, aa = self._arrays(batches)
        w = self.window.c()
        nb = len(bs)
        self.reserve(self.workspace_bytes(batches))
        if groups is None:
            slide = self.window.slide or self.window.length
            per = -(-self.window.length // slide)
            caps = caps or [b.batch.nrows * per for b in bs]
            groups = [Groups(c, self.aggs, self.device) for c in caps]
        if d_counts is None:
            d_counts = torch.zeros((nb, 2), dtype=torch.int64, device=self.device)
        outs = (lms_groups * nb)(*[g.c for g in groups])
        pa, npred = _preds(self.preds)
        pr, nproj = _projs(self.projs)
        _check(_lib.lms_window_agg_multi_prepare(arr, nb, pa, npred, pr, nproj, self.key_col, ctypes.byref(w), aa,
                                                 len(self.aggs), outs, d_counts.data_ptr(), self.ws.data_ptr(),
                                                 self.ws.numel(), ctypes.byref(self.cfg), _stream_handle(stream)))
        self._keep = (bs, groups, d_counts)
        self.groups, self.d_counts = groups, d_counts
        return groups, d_counts

    def launch(self, stream=None, cfg: lms_multi_config | None = None):
        c = cfg or self.launch_cfg or self.cfg
        _check(_lib.lms_window_agg_multi_launch(ctypes.byref(c), self.ws.data_ptr(), _stream_handle(stream)))

    def freeze(self, max_nparts=None):
        """Fixes the launch configuration and the workspace (as for graph capture) to
        the prepared ones, or with room for up to ``max_nparts`` partitions per batch.
        Later prepares must fit the workspace; jobs beyond the launch limits are
        rejected by the kernels (status LMS_EINVAL)."""
        c = lms_multi_config()
        ctypes.pointer(c)[0] = self.cfg
        if max_nparts:
            c.max_nparts = max(c.max_nparts, max_nparts)
        self.launch_cfg = c
        return c


def lms_window_agg_multi(batches, key_col, window: Window, aggs, preds=(), projs=(), stream=None):
    """One-shot multi-batch windowed group-by; returns (list of Groups, d_counts[nb, 2])."""
    job = MultiJob(key_col, window, aggs, preds, projs, device=batches[0][0].device)
    g, d = job.prepare(batches, stream=stream)
    job.launch(stream=stream)
    return g, d, job


class WindowState:
    """Device-resident partial aggregates of a windowed group-by over a stream of
    micro-batches (lms_wstate_*): ``update`` adds a batch, ``emit`` writes the
    windows the watermark has closed (all remaining ones with ``flush``)."""

    INFO = ("late_rows", "dropped_rows", "min_pane", "max_pane", "next_window", "emit_lo", "emit_hi", "status")

    def __init__(self, window: Window, aggs, max_keys: int, ring_panes: int = 32, device=None, stream=None):
        self.window, self.aggs = window, list(aggs)
        self.device = device or torch.device("cuda")
        aa = (lms_agg * max(1, len(self.aggs)))(*[lms_agg(f, c) for f, c in self.aggs])
        w = window.c()
        h = ctypes.c_void_p()
        _check(_lib.lms_wstate_create(ctypes.byref(w), aa, len(self.aggs), max_keys, ring_panes, ctypes.byref(h),
                                      _stream_handle(stream)))
        self.handle = h
        self.nbytes = int(_lib.lms_wstate_bytes(max_keys, ring_panes, len(self.aggs)))
        self._info = torch.zeros(8, dtype=torch.int64, device=self.device)

    @staticmethod
    def bytes(max_keys: int, ring_panes: int, nagg: int) -> int:
        return int(_lib.lms_wstate_bytes(max_keys, ring_panes, nagg))

    def update(self, cols, key_col, preds=(), projs=(), stream=None):
        b = _Batch(cols)
        pa, npred = _preds(preds)
        pr, nproj = _projs(projs)
        _check(_lib.lms_wstate_update(self.handle, ctypes.byref(b.batch), pa, npred, pr, nproj, key_col,
                                      _stream_handle(stream)))
        return b  # keeps the column array alive until the caller drops it

    def emit(self, watermark: int = 0, flush: bool = False, max_windows: int = 1 << 20, groups=None, cap=None,
             d_count=None, stream=None):
        if groups is None:
            groups = Groups(cap if cap is not None else 1 << 16, self.aggs, self.device)
        if d_count is None:
            d_count = torch.zeros(2, dtype=torch.int64, device=self.device)
        _check(_lib.lms_wstate_emit(self.handle, int(watermark), int(bool(flush)), int(max_windows),
                                    ctypes.byref(groups.c), d_count.data_ptr(), _stream_handle(stream)))
        return groups, d_count

    def info(self, stream=None) -> dict:
        _check(_lib.lms_wstate_info(self.handle, self._info.data_ptr(), _stream_handle(stream)))
        return dict(zip(self.INFO, (int(x) for x in self._info.cpu())))

    def free(self):
        if self.handle:
            _lib.lms_wstate_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Admission:
    """ConstructMicroBatch (lms_admit_*): buffers arriving datasets and decides at
    each poll whether they form the next micro-batch."""

    def __init__(self, slide_ms=0.0, deadline_ms=0.0, poll_ms=10.0, poll_idle=True):
        p = lms_admit_params(float(slide_ms), float(deadline_ms), float(poll_ms), int(bool(poll_idle)), 0)
        h = ctypes.c_void_p()
        _check(_lib.lms_admit_create(ctypes.byref(p), ctypes.byref(h)))
        self.handle = h
        self._d = lms_admit_decision()

    def poll(self, now_ms, arrival_ms=(), rows=()) -> lms_admit_decision:
        import numpy as np
        a = np.ascontiguousarray(arrival_ms, dtype=np.float64)
        r = np.ascontiguousarray(rows, dtype=np.int64)
        if len(a) != len(r):
            raise ValueError("arrival_ms and rows differ in length")
        _check(_lib.lms_admit_poll(self.handle, float(now_ms), len(a), a.ctypes.data, r.ctypes.data,
                                   ctypes.byref(self._d)))
        return self._d

    def done(self, rows, proc_ms, maxlat_ms):
        _check(_lib.lms_admit_done(self.handle, int(rows), float(proc_ms), float(maxlat_ms)))

    def set_model(self, model, ops, selectivity=1.0, distinct_keys=0, num_cores=1, interval_s=0.0,
                  bytes_per_row=24.0):
        """Learned sizing: Eq. 6's processing term from the learned cost model.

        ops: [(kind, ncols, window_s, slide_s)] of the query's operation chain;
        model None returns to Eq. 4's AvgThPut."""
        import numpy as np
        if model is None:
            _check(_lib.lms_admit_set_model(self.handle, None, None, 0, None, 0.0))
            return
        keep = np.ascontiguousarray(model, dtype=np.float32)
        if keep.size != MLP_NPARAMS:
            raise ValueError("model must hold MLP_NPARAMS float32 parameters")
        arr = (lms_op_desc * len(ops))(*[lms_op_desc(int(k), int(c), 0.0, float(w), float(sl)) for k, c, w, sl in ops])
        st = lms_batch_stats(0, int(num_cores), 0, 0, float(selectivity), int(distinct_keys), float(interval_s))
        _check(_lib.lms_admit_set_model(self.handle, keep.ctypes.data, arr, len(ops), ctypes.byref(st),
                                        float(bytes_per_row)))

    def predict_ms(self, rows) -> float:
        return float(_lib.lms_admit_predict_ms(self.handle, int(rows)))

    def stats(self) -> dict:
        st = lms_admit_stats()
        _check(_lib.lms_admit_get_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in lms_admit_stats._fields_}

    def __del__(self):
        try:
            if self.handle:
                _lib.lms_admit_free(self.handle)
                self.handle = None
        except Exception:
            pass


def set_tuning(chunk_rows=0, part_rows=0, piece_rows=0, grid_per_cu=0, lds_groups=0):
    t = lms_tuning(chunk_rows, part_rows, piece_rows, grid_per_cu, lds_groups, 0)
    _check(_lib.lms_set_tuning(ctypes.byref(t)))


def get_tuning() -> dict:
    t = lms_tuning()
    _check(_lib.lms_get_tuning(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in lms_tuning._fields_ if f != "reserved"}


# ---- stream-static join ------------------------------------------------------------------

class JoinTable:
    def __init__(self, handle: int, keys: torch.Tensor, payload: torch.Tensor):
        self.handle = ctypes.c_void_p(handle)
        self._keep = (keys, payload)  # inputs stay alive until the build completed

    def max_mult(self) -> int:
        m = int(_lib.lms_join_max_mult(self.handle))
        if m < 0:
            raise LmsError(m, last_error())
        return m

    def free(self):
        if self.handle:
            _lib.lms_join_free(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lms_join_build(keys: torch.Tensor, payload: torch.Tensor, stream=None) -> JoinTable:
    b = _Batch([keys, payload])
    h = ctypes.c_void_p(0)
    rc = _lib.lms_join_build(ctypes.byref(b.batch), 0, 1, ctypes.byref(h), _stream_handle(stream))
    _check(rc)
    return JoinTable(h.value, keys, payload)


def lms_hash_join(table: JoinTable, probe_keys: torch.Tensor, cap: int | None = None, out=None, d_count=None,
                  workspace=None, stream=None):
    """Enqueues the probe; returns (probe_idx uint32 as int32 tensor, payload, d_count)."""
    b = _Batch([probe_keys])
    n = b.batch.nrows
    dev = probe_keys.device
    if cap is None:
        cap = n * max(1, table.max_mult())
    if out is None:
        out = (torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
               torch.empty(max(cap, 1), dtype=torch.int32, device=dev))
    if d_count is None:
        d_count = torch.zeros(2, dtype=torch.int64, device=dev)
    need = _lib.lms_hash_join_workspace(n)
    ws = _ws(workspace, need, dev, stream)
    rc = _lib.lms_hash_join(table.handle, ctypes.byref(b.batch), 0, out[0].data_ptr(), out[1].data_ptr(), cap,
                            d_count.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream))
    _check(rc)
    return out[0], out[1], d_count


# ---- CPU execution functions (host tensors, synchronous) -------------------------------------

def lms_cpu_filter_project(cols, preds=(), keep=(), projs=(), nthreads=1):
    """Filter + project on host tensors; returns the trimmed output columns."""
    b = _Batch(cols)
    n = b.batch.nrows
    keep, projs = list(keep), list(projs)
    out = [torch.empty(n, dtype=cols[c].dtype) for c in keep] + [torch.empty(n, dtype=cols[p[0]].dtype) for p in projs]
    ob = _Batch(out, nrows=n)
    pa, npred = _preds(preds)
    pr, nproj = _projs(projs)
    ka = (ctypes.c_int32 * max(1, len(keep)))(*keep)
    cnt = ctypes.c_int64(0)
    _check(_lib.lms_cpu_filter_project(ctypes.byref(b.batch), pa, npred, ka, len(keep), pr, nproj,
                                       ctypes.byref(ob.batch), ctypes.byref(cnt), nthreads))
    return [o[:cnt.value] for o in out]


def lms_cpu_window_agg(cols, key_col, window: "Window", aggs, preds=(), projs=(), cap=None, nthreads=1):
    """Windowed group-by on host tensors; returns (key, wstart, [aggs]) trimmed to the group count."""
    b = _Batch(cols)
    n = b.batch.nrows
    aggs = list(aggs)
    if cap is None:
        slide = window.slide or window.length
        cap = n * (-(-window.length // slide))
    g = Groups(cap, aggs, torch.device("cpu"))
    pa, npred = _preds(preds)
    pr, nproj = _projs(projs)
    aa = (lms_agg * max(1, len(aggs)))(*[lms_agg(f, c) for f, c in aggs])
    w = window.c()
    cnt = ctypes.c_int64(0)
    _check(_lib.lms_cpu_window_agg(ctypes.byref(b.batch), pa, npred, pr, nproj, key_col, ctypes.byref(w), aa,
                                   len(aggs), ctypes.byref(g.c), ctypes.byref(cnt), nthreads))
    m = min(cnt.value, cap)
    return g.key[:m], g.wstart[:m], [a[:m] for a in g.aggs], cnt.value


def lms_cpu_hash_join(build_keys, build_payload, probe_keys, cap=None, nthreads=1):
    """Join on host tensors; returns (probe_idx int32 view of uint32, payload, count)."""
    tb = _Batch([build_keys, build_payload])
    pb = _Batch([probe_keys])
    if cap is None:
        cap = max(1, int(probe_keys.shape[0]) * 4)
    oi = torch.empty(cap, dtype=torch.int32)
    op = torch.empty(cap, dtype=torch.int32)
    cnt = ctypes.c_int64(0)
    _check(_lib.lms_cpu_hash_join(ctypes.byref(tb.batch), 0, 1, ctypes.byref(pb.batch), 0, oi.data_ptr(),
                                  op.data_ptr(), cap, ctypes.byref(cnt), nthreads))
    m = min(cnt.value, cap)
    return oi[:m], op[:m], cnt.value


# ---- kernel tracing ----------------------------------------------------------------------

def lms_trace_enable(on: bool = True):
    _check(_lib.lms_trace_enable(1 if on else 0))


def lms_trace_read() -> dict:
    """Per-kernel {name: (launches, total_ms, min_ms, max_ms)} since the last read (synchronises)."""
    buf = (lms_trace_stat * 64)()
    n = _lib.lms_trace_read(buf, 64)
    if n < 0:
        raise LmsError(n, last_error())
    return {buf[i].name.decode(): (int(buf[i].launches), buf[i].total_ms, buf[i].min_ms, buf[i].max_ms)
            for i in range(min(n, 64))}


# ---- placement --------------------------------------------------------------------------

def table2_base_cost(kind: int) -> float:
    return float(_lib.lms_table2_base_cost(kind))


def lms_plan(kinds, batch_bytes, num_cores, infpt_bytes=150.0 * 1024, base_trans=0.1, base_costs=None,
             rows=0, selectivity=1.0, distinct_keys=0, mode=PLAN_ANALYTIC, model=None, ncols=None, window_s=None,
             slide_s=None, interval_s=0.0):
    """MapDevice (Algorithm 2) over the chain `kinds`; returns (devices, costs).

    model: float32 array of the MLP's parameters (LMS_PLAN_LEARNED mode)."""
    kinds = list(kinds)
    n = len(kinds)
    ops = (lms_op_desc * max(1, n))()
    for i, k in enumerate(kinds):
        ops[i] = lms_op_desc(k, int(ncols[i]) if ncols is not None else 1,
                             float(base_costs[i]) if base_costs is not None else 0.0,
                             float(window_s[i]) if window_s is not None else 0.0,
                             float(slide_s[i]) if slide_s is not None else 0.0)
    st = lms_batch_stats(int(batch_bytes), int(num_cores), 0, int(rows), float(selectivity), int(distinct_keys),
                         float(interval_s))
    keep = None
    mp = None
    if model is not None:
        import numpy as np
        keep = np.ascontiguousarray(model, dtype=np.float32)
        if keep.size != MLP_NPARAMS:
            raise ValueError("model must hold MLP_NPARAMS float32 parameters")
        mp = keep.ctypes.data
    cp = lms_cost_params(float(infpt_bytes), float(base_trans), mode, 0, mp)
    dev = (ctypes.c_int32 * max(1, n))()
    cost = (ctypes.c_double * max(1, n))()
    _check(_lib.lms_plan(ops, n, ctypes.byref(st), ctypes.byref(cp), dev, cost))
    return list(dev)[:n], list(cost)[:n]


class InfPTTuner:
    """Eq. 10: online regression of the inflection point (lms_infpt_*)."""

    def __init__(self, init_bytes=150.0 * 1024, history=0, jitter=0.1, seed=0):
        h = ctypes.c_void_p()
        _check(_lib.lms_infpt_create(float(init_bytes), int(history), float(jitter), int(seed), ctypes.byref(h)))
        self.handle = h

    def record(self, infpt_used, thput, maxlat):
        _check(_lib.lms_infpt_record(self.handle, float(infpt_used), float(thput), float(maxlat)))

    def next(self, target_latency=0.0) -> float:
        return float(_lib.lms_infpt_next(self.handle, float(target_latency)))

    def __del__(self):
        try:
            if self.handle:
                _lib.lms_infpt_free(self.handle)
                self.handle = None
        except Exception:
            pass


# ---- learned placement model -------------------------------------------------------------

MLP_NPARAMS = 64 * 12 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def mlp_features(kind, rows, ncols, selectivity, distinct_keys, window_s, slide_s, interval_s, transfer):
    """The model's 12 input features of one operation (the library's definition)."""
    import numpy as np
    op = lms_op_desc(kind, int(ncols), 0.0, float(window_s), float(slide_s))
    st = lms_batch_stats(0, 1, 0, int(rows), float(selectivity), int(distinct_keys), float(interval_s))
    x = np.zeros(12, np.float32)
    _lib.lms_mlp_features(ctypes.byref(op), ctypes.byref(st), int(transfer), x.ctypes.data)
    return x


class Mlp:
    """Device copy of the placement MLP with its Adam state."""

    def __init__(self, seed: int = 0, device=None):
        self.device = device or torch.device("cuda")
        h = ctypes.c_void_p(0)
        _check(_lib.lms_mlp_create(int(seed), ctypes.byref(h)))
        self.h = h
        self.grad = torch.zeros(MLP_NPARAMS, dtype=torch.float32, device=self.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.ws = Workspace(self.device)

    def set_params(self, p):
        import numpy as np
        a = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.lms_mlp_set_params(self.h, a.ctypes.data))

    def get_params(self):
        import numpy as np
        a = np.zeros(MLP_NPARAMS, np.float32)
        _check(_lib.lms_mlp_get_params(self.h, a.ctypes.data))
        return a

    def loss_grad_async(self, X, T, M, stream=None):
        n = int(X.shape[0])
        ws = self.ws.get(_lib.lms_mlp_workspace(n))
        _check(_lib.lms_mlp_loss_grad(self.h, X.data_ptr(), T.data_ptr(), M.data_ptr(), n, self.grad.data_ptr(),
                                      self.loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)))

    def loss_grad(self, X, T, M, stream=None):
        """Loss (float) and gradient (numpy) of the masked squared error (synchronises)."""
        self.loss_grad_async(X, T, M, stream)
        torch.cuda.synchronize()
        return float(self.loss.item()), self.grad.cpu().numpy()

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(_lib.lms_mlp_adam_step(self.h, self.grad.data_ptr(), lr, beta1, beta2, eps, _stream_handle(stream)))

    def forward(self, X, bf16=False, stream=None):
        n = int(X.shape[0])
        y = torch.empty(max(n, 1), 2, dtype=torch.float32, device=self.device)
        _check(_lib.lms_mlp_forward(self.h, X.data_ptr(), n, y.data_ptr(), 1 if bf16 else 0, _stream_handle(stream)))
        return y[:n]

    def free(self):
        if self.h:
            _lib.lms_mlp_free(self.h)
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

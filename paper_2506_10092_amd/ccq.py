"""ctypes binding for libccq (include/ccq.h): argument marshalling only.

Device memory and streams come from torch; every step of a query runs in the
library's HIP kernels.  The binding refuses to work when libccq.so is
missing -- there is no CPU fallback.

Column dicts follow the generator's format (see ``datagen``) but hold torch
tensors on the GPU::

    {"enc": "rle", "values": int32|int64, "run_ends": int64}
    {"enc": "index", "positions": int32|int64, "values": int32|int64}
    {"enc": "bitpacked", "packed": int32 (the uint32 words), "w": int, "base": int}

A query names columns and uses the same dict layout as the generator::

    {"preds": [(col, "range" | "not_range", lo, hi) | (col, "in" | "not_in", [...])],
     "or": [[pred, pred, ...], ...],
     "keys": [(col, shift, card)], "aggs": [("count",) | ("sum", col)],
     "window": (row_begin, row_end)}

The filter is every entry of "preds" ANDed with every clause of "or" (optional),
a clause being the OR of its predicates.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccq.so")

OK, E_INVALID, E_UNSUPPORTED, E_CAPACITY, E_KEY_DOMAIN, E_HIP, E_BUDGET, E_BUSY, E_NOMEM = 0, -1, -2, -3, -4, -5, -6, -7, -8
RLE, INDEX, BITPACKED, RLE_INDEX, PLAIN_INDEX = 1, 2, 3, 4, 5
I32, I64 = 1, 2
RANGE, IN, NOT_RANGE, NOT_IN = 1, 2, 3, 4
COUNT_STAR, SUM, MIN, MAX = 1, 2, 3, 4
OPS = {"+": 1, "-": 2, "*": 3}
HOST_ONLY = -1
# size of the fixed device scratch ccq_execute_noalloc uses as the workspace (include/ccq.h)
NOALLOC_WORKSPACE_BYTES = 32 << 20

_STATUS_NAMES = {0: "CCQ_OK", -1: "CCQ_E_INVALID", -2: "CCQ_E_UNSUPPORTED", -3: "CCQ_E_CAPACITY",
                 -4: "CCQ_E_KEY_DOMAIN", -5: "CCQ_E_HIP", -6: "CCQ_E_BUDGET", -7: "CCQ_E_BUSY", -8: "CCQ_E_NOMEM"}


class CcqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, str(status)), msg))
        self.status = status


class ColumnDesc(ctypes.Structure):
    _fields_ = [("encoding", ctypes.c_int32), ("value_type", ctypes.c_int32), ("n_entries", ctypes.c_int64),
                ("values", ctypes.c_void_p), ("run_ends", ctypes.c_void_p), ("positions", ctypes.c_void_p),
                ("packed", ctypes.c_void_p), ("bit_width", ctypes.c_int32), ("position_type", ctypes.c_int32),
                ("base", ctypes.c_int64), ("dict_values", ctypes.c_void_p), ("dict_size", ctypes.c_int64),
                ("point_values", ctypes.c_void_p), ("n_points", ctypes.c_int64)]


class Pred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("op", ctypes.c_int32), ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
                ("in_list", ctypes.c_void_p), ("in_len", ctypes.c_int64), ("clause", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class Key(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("shift", ctypes.c_int32), ("card", ctypes.c_int64)]


class Agg(ctypes.Structure):
    _fields_ = [("func", ctypes.c_int32), ("col", ctypes.c_int32), ("op", ctypes.c_int32), ("col2", ctypes.c_int32)]


class QueryDesc(ctypes.Structure):
    _fields_ = [("preds", ctypes.POINTER(Pred)), ("n_preds", ctypes.c_int32),
                ("keys", ctypes.POINTER(Key)), ("n_keys", ctypes.c_int32),
                ("aggs", ctypes.POINTER(Agg)), ("n_aggs", ctypes.c_int32),
                ("row_begin", ctypes.c_int64), ("row_end", ctypes.c_int64)]


class ExecOpts(ctypes.Structure):
    _fields_ = [("fused_begin", ctypes.c_void_p), ("fused_end", ctypes.c_void_p)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("tiles_per_item", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("n_streams", ctypes.c_int32), ("batching", ctypes.c_int32),
                ("tiles_per_item", ctypes.c_int32), ("no_graphs", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class ResultDesc(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("counts", ctypes.c_void_p), ("aggs", ctypes.c_void_p),
                ("n_groups", ctypes.c_void_p), ("status", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class EncodingChoice(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("runs", ctypes.c_int64), ("single_runs", ctypes.c_int64),
                ("min_value", ctypes.c_int64), ("max_value", ctypes.c_int64), ("lo_cut", ctypes.c_int64),
                ("hi_cut", ctypes.c_int64), ("choice", ctypes.c_int32), ("bit_width", ctypes.c_int32),
                ("base", ctypes.c_int64), ("rle_runs", ctypes.c_int64), ("index_points", ctypes.c_int64)]


CHOICE_NAMES = {1: "plain", 2: "rle", 3: "rle+index", 4: "plain+index"}


# every function include/ccq.h declares: name -> (restype, argtypes)
_vp, _i32, _i64, _sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
SIGNATURES = {
    "ccq_last_error": (ctypes.c_char_p, []),
    "ccq_abi_version": (_i32, []),
    "ccq_context_create": (_i32, [_i32, ctypes.POINTER(_vp)]),
    "ccq_context_destroy": (None, [_vp]),
    "ccq_table_create": (_i32, [_vp, _i64, ctypes.POINTER(ColumnDesc), _i32, ctypes.POINTER(_vp)]),
    "ccq_table_destroy": (None, [_vp]),
    "ccq_table_validate": (_i32, [_vp, _vp]),
    "ccq_plan_check": (_i32, [_vp, ctypes.POINTER(QueryDesc), ctypes.POINTER(_i64), ctypes.POINTER(_sz)]),
    "ccq_plan_create": (_i32, [_vp, ctypes.POINTER(QueryDesc), ctypes.POINTER(_vp)]),
    "ccq_plan_destroy": (None, [_vp]),
    "ccq_plan_info": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_sz)]),
    "ccq_execute": (_i32, [_vp, _vp, _sz, _vp, ctypes.POINTER(ResultDesc)]),
    "ccq_execute_ex": (_i32, [_vp, _vp, _sz, _vp, ctypes.POINTER(ResultDesc), ctypes.POINTER(ExecOpts)]),
    "ccq_execute_noalloc": (_i32, [_vp, _vp, ctypes.POINTER(ResultDesc)]),
    "ccq_batch_create": (_i32, [_vp, ctypes.POINTER(_vp), _i32, ctypes.POINTER(ResultDesc), ctypes.POINTER(BatchOpts),
                                ctypes.POINTER(_vp)]),
    "ccq_batch_destroy": (None, [_vp]),
    "ccq_batch_info": (_i32, [_vp, ctypes.POINTER(_sz), ctypes.POINTER(_i64)]),
    "ccq_batch_set_tiles_per_item": (_i32, [_vp, _i32]),
    "ccq_batch_execute": (_i32, [_vp, _vp, _sz, _vp]),
    "ccq_batch_execute_ex": (_i32, [_vp, _vp, _sz, _vp, ctypes.POINTER(ExecOpts)]),
    "ccq_batch_autotune": (_i32, [_vp, _vp, _sz, _vp, ctypes.POINTER(_i32), _i32, _i32, ctypes.POINTER(_i32),
                                  ctypes.POINTER(ctypes.c_float)]),
    "ccq_now": (ctypes.c_double, []),
    "ccq_server_create": (_i32, [_vp, ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    "ccq_server_submit": (_i32, [_vp, _vp, ctypes.POINTER(ResultDesc), ctypes.POINTER(ctypes.c_uint64)]),
    "ccq_server_poll": (_i32, [_vp, ctypes.POINTER(Completion), _i32, ctypes.POINTER(_i32)]),
    "ccq_server_drain": (_i32, [_vp, ctypes.c_double]),
    "ccq_server_destroy": (None, [_vp]),
    "ccq_avg_var": (_i32, [_vp, _vp, _vp, _i64, _vp, _vp]),
    "ccq_encode_workspace_bytes": (_sz, [_i64]),
    "ccq_encode_choose": (_i32, [_vp, _vp, _i32, _i64, _vp, _sz, _vp, ctypes.POINTER(EncodingChoice)]),
    "ccq_plain_to_rle": (_i32, [_vp, _vp, _i32, _i64, _vp, _sz, _vp, _vp, _vp, _i64, ctypes.POINTER(_i64)]),
    "ccq_plain_to_rle_index": (_i32, [_vp, _vp, _i32, _i64, _vp, _sz, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _i64,
                                      ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "ccq_plain_to_plain_index": (_i32, [_vp, _vp, _i32, _i64, _i32, _i64, _vp, _sz, _vp, _vp, _i64, _vp, _vp, _i64,
                                        ctypes.POINTER(_i64)]),
    "ccq_tune_cache_load": (_i32, [_vp, ctypes.c_char_p, ctypes.POINTER(_i64)]),
    "ccq_tune_cache_save": (_i32, [_vp, ctypes.c_char_p, ctypes.POINTER(_i64)]),
    "ccq_join_workspace_bytes": (_sz, [_vp, _i32, _i64, _i64, _vp, _i32, _i64, _i64]),
    "ccq_join_index": (_i32, [_vp, _i32, _i64, _i64, _vp, _i32, _i64, _i64, _vp, _sz, _vp, _vp, _i64,
                              ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "ccq_join_apply_workspace_bytes": (_sz, [_i64, _i64]),
    "ccq_join_apply": (_i32, [_vp, _i32, _vp, _i64, _i32, _vp, _sz, _vp, _vp, _i64, ctypes.POINTER(_i64)]),
}

_lib = None


def lib():
    """Load libccq.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        # torch carries its own HIP runtime; loading it first makes this
        # library bind to that same runtime, so device pointers and streams
        # from torch are valid here (one runtime per process)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise CcqError(E_UNSUPPORTED, "libccq.so is not built (run __graft_entry__.build()); "
                                          "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != OK:
        raise CcqError(status, lib().ccq_last_error().decode())


def _dtype_code(t):
    import torch
    if t.dtype == torch.int32:
        return I32
    if t.dtype == torch.int64:
        return I64
    raise CcqError(E_INVALID, "values must be int32 or int64 tensors, got %s" % t.dtype)


class Context:
    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(lib().ccq_context_create(int(device), ctypes.byref(h)))
        self.h = h
        self.device = device

    def tune_cache_load(self, path):
        """Merge a tuning-cache file into this context's cache; returns the entries read."""
        n = ctypes.c_int64()
        _check(lib().ccq_tune_cache_load(self.h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def tune_cache_save(self, path):
        """Write this context's tuning cache to `path`; returns the entries written."""
        n = ctypes.c_int64()
        _check(lib().ccq_tune_cache_save(self.h, os.fsencode(path), ctypes.byref(n)))
        return n.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ccq_context_destroy(self.h)
            self.h = None


def _column_desc(c, n_rows):
    """Column dict -> ccq_column_desc.  Composites: "rle+index" {values,
    run_ends (the last equal to n_rows; a run stands for the rows from the
    previous end that no point lists), positions, point_values}; "plain+index"
    {packed, w, base, positions, point_values}."""
    d = ColumnDesc()
    if c["enc"] in ("rle+index", "plain+index"):
        base = dict(c, enc="rle" if c["enc"] == "rle+index" else "bitpacked")
        for k in ("positions", "point_values"):
            base.pop(k, None)
        d = _column_desc(base, n_rows)
        d.encoding = RLE_INDEX if c["enc"] == "rle+index" else PLAIN_INDEX
        pv = c["point_values"]
        if c["enc"] == "plain+index":
            d.value_type = _dtype_code(pv)
        elif _dtype_code(pv) != d.value_type:
            raise CcqError(E_INVALID, "run values and point values must share one type")
        d.position_type = _dtype_code(c["positions"])
        d.positions, d.point_values, d.n_points = c["positions"].data_ptr(), pv.data_ptr(), pv.numel()
        return d
    if c["enc"] == "rle":
        d.encoding, d.value_type, d.n_entries = RLE, _dtype_code(c["values"]), c["run_ends"].numel()
        d.values, d.run_ends = c["values"].data_ptr(), c["run_ends"].data_ptr()
    elif c["enc"] == "index":
        d.encoding, d.value_type, d.n_entries = INDEX, _dtype_code(c["values"]), c["positions"].numel()
        d.position_type = _dtype_code(c["positions"])
        d.values, d.positions = c["values"].data_ptr(), c["positions"].data_ptr()
    elif c["enc"] == "bitpacked":
        d.encoding, d.n_entries, d.bit_width, d.base = BITPACKED, n_rows, int(c["w"]), int(c.get("base", 0))
        d.packed = c["packed"].data_ptr()
        if c.get("dict") is not None:      # int64 dictionary tensor (device)
            d.dict_values, d.dict_size = c["dict"].data_ptr(), c["dict"].numel()
    else:
        raise CcqError(E_INVALID, "unknown encoding %r" % (c["enc"],))
    return d


class Table:
    """Encoded columns (device tensors, borrowed) over n_rows logical rows."""

    def __init__(self, ctx, n_rows, columns):
        self.ctx = ctx
        self.n_rows = int(n_rows)
        self.names = list(columns)
        self.columns = columns            # keeps the tensors alive
        arr = (ColumnDesc * max(len(self.names), 1))()
        for i, n in enumerate(self.names):
            arr[i] = _column_desc(columns[n], self.n_rows)
        h = ctypes.c_void_p()
        _check(lib().ccq_table_create(ctx.h, self.n_rows, arr, len(self.names), ctypes.byref(h)))
        self.h = h

    def validate(self, stream=None):
        _check(lib().ccq_table_validate(self.h, _stream_ptr(stream)))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ccq_table_destroy(self.h)
            self.h = None


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _event_handle(ev, stream):
    """Raw hipEvent_t of a torch.cuda.Event (created lazily by torch, so
    record it once first)."""
    if not ev.cuda_event:
        ev.record() if stream is None else ev.record(stream)
    return ctypes.c_void_p(ev.cuda_event)


def query_desc(table, query):
    """Marshal a query dict into a QueryDesc; returns (desc, keepalive)."""
    idx = {n: i for i, n in enumerate(table.names)}

    def col(name):
        if name not in idx:
            raise CcqError(E_INVALID, "unknown column %r" % (name,))
        return idx[name]

    keep = []
    flat = [(p, 0) for p in query["preds"]]
    for k, clause in enumerate(query.get("or", ())):
        if not clause:
            raise CcqError(E_INVALID, "OR clause %d is empty" % k)
        flat += [(p, k + 1) for p in clause]
    preds = (Pred * max(len(flat), 1))()
    for i, (p, clause) in enumerate(flat):
        preds[i].col = col(p[0])
        preds[i].clause = clause
        if p[1] in ("range", "not_range"):
            preds[i].op = RANGE if p[1] == "range" else NOT_RANGE
            preds[i].lo, preds[i].hi = int(p[2]), int(p[3])
        elif p[1] in ("in", "not_in"):
            lst = np.ascontiguousarray(np.array(list(p[2]), dtype=np.int64))
            keep.append(lst)
            preds[i].op = IN if p[1] == "in" else NOT_IN
            preds[i].in_list, preds[i].in_len = lst.ctypes.data, len(lst)
        else:
            raise CcqError(E_INVALID, "unknown predicate %r" % (p[1],))
    keys = (Key * max(len(query["keys"]), 1))()
    for i, k in enumerate(query["keys"]):
        keys[i].col, keys[i].shift, keys[i].card = col(k[0]), int(k[1]), int(k[2])
    aggs = (Agg * max(len(query["aggs"]), 1))()
    for i, a in enumerate(query["aggs"]):
        if a[0] == "count":
            aggs[i].func, aggs[i].col = COUNT_STAR, -1
        elif a[0] in ("sum", "min", "max"):
            aggs[i].func = {"sum": SUM, "min": MIN, "max": MAX}[a[0]]
            if isinstance(a[1], tuple):        # (col, op, col2): the row-wise col op col2
                if a[1][1] not in OPS:
                    raise CcqError(E_INVALID, "unknown operator %r" % (a[1][1],))
                aggs[i].col, aggs[i].op, aggs[i].col2 = col(a[1][0]), OPS[a[1][1]], col(a[1][2])
            else:
                aggs[i].col = col(a[1])
        else:
            raise CcqError(E_INVALID, "unknown aggregate %r" % (a[0],))
    rb, re_ = query.get("window", (0, table.n_rows))
    d = QueryDesc(preds, len(flat), keys, len(query["keys"]), aggs, len(query["aggs"]), int(rb), int(re_))
    keep += [preds, keys, aggs]
    return d, keep


def plan_check(table, query):
    """Validate and compile without allocating: (max_groups, workspace_bytes)."""
    d, keep = query_desc(table, query)
    g, w = ctypes.c_int64(), ctypes.c_size_t()
    _check(lib().ccq_plan_check(table.h, ctypes.byref(d), ctypes.byref(g), ctypes.byref(w)))
    return g.value, w.value


class Result:
    """Caller-owned device result buffers."""

    def __init__(self, capacity, n_keys, n_aggs, device):
        import torch
        self.capacity = int(capacity)
        self.n_keys, self.n_aggs = n_keys, n_aggs
        self.keys = torch.zeros(max(self.capacity * n_keys, 1), dtype=torch.int64, device=device)
        self.counts = torch.zeros(max(self.capacity, 1), dtype=torch.int64, device=device)
        self.aggs = torch.zeros(max(self.capacity * n_aggs, 1), dtype=torch.int64, device=device)
        self.n_groups = torch.zeros(1, dtype=torch.int64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.desc = ResultDesc(self.keys.data_ptr(), self.counts.data_ptr(), self.aggs.data_ptr(),
                               self.n_groups.data_ptr(), self.status.data_ptr(), self.capacity)

    def to_python(self):
        """Copy to host (synchronises) and return {"keys", "counts", "aggs", "status"}."""
        g = int(self.n_groups.item())
        st = int(self.status.item())
        nk, na = self.n_keys, self.n_aggs
        k = self.keys[: g * nk].cpu().numpy().reshape(g, nk) if nk else np.zeros((g, 0), dtype=np.int64)
        c = self.counts[:g].cpu().numpy()
        a = self.aggs[: g * na].cpu().numpy().reshape(g, na) if na else np.zeros((g, 0), dtype=np.int64)
        return {"keys": [tuple(int(x) for x in row) for row in k], "counts": [int(x) for x in c],
                "aggs": [tuple(int(x) for x in row) for row in a], "status": st}


class Plan:
    def __init__(self, table, query):
        self.table = table
        self.query = query
        d, keep = query_desc(table, query)
        h = ctypes.c_void_p()
        _check(lib().ccq_plan_create(table.h, ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        g, w = ctypes.c_int64(), ctypes.c_size_t()
        _check(lib().ccq_plan_info(h, ctypes.byref(g), ctypes.byref(w)))
        self.max_groups, self.workspace_bytes = g.value, w.value
        self.n_keys, self.n_aggs = len(query["keys"]), len(query["aggs"])

    def new_workspace(self):
        import torch
        # torch's caching allocator returns 512-byte aligned blocks
        return torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device="cuda:%d" % self.table.ctx.device)

    def new_result(self):
        return Result(self.max_groups, self.n_keys, self.n_aggs, "cuda:%d" % self.table.ctx.device)

    def execute(self, workspace, result, stream=None, fused_events=None):
        """Enqueue the query on `stream` (torch stream, raw handle or None =
        current).  fused_events: optional (begin, end) torch.cuda.Event pair
        recorded around the fused kernel on that stream."""
        if fused_events is None:
            _check(lib().ccq_execute(self.h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                     _stream_ptr(stream), ctypes.byref(result.desc)))
            return
        opts = ExecOpts(_event_handle(fused_events[0], stream), _event_handle(fused_events[1], stream))
        _check(lib().ccq_execute_ex(self.h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                    _stream_ptr(stream), ctypes.byref(result.desc), ctypes.byref(opts)))

    def execute_noalloc(self, result, stream=None):
        """Enqueue the query on `stream` with the library's fixed device
        scratch as its workspace (ccq_execute_noalloc)."""
        _check(lib().ccq_execute_noalloc(self.h, _stream_ptr(stream), ctypes.byref(result.desc)))

    def run(self):
        """Execute once and return the result on the host."""
        ws, res = self.new_workspace(), self.new_result()
        self.execute(ws, res)
        return res.to_python()

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ccq_plan_destroy(self.h)
            self.h = None


class Batch:
    """Many plans in one launch sequence (ccq_batch_*); results land in one
    Result per plan, fixed at creation."""

    def __init__(self, ctx, plans, tiles_per_item=0, use_graph=False):
        self.ctx = ctx
        self.plans = list(plans)
        self.results = [p.new_result() for p in self.plans]
        n = len(self.plans)
        parr = (ctypes.c_void_p * max(n, 1))(*[p.h.value for p in self.plans])
        rarr = (ResultDesc * max(n, 1))()
        for i, r in enumerate(self.results):
            rarr[i] = r.desc
        opts = BatchOpts(int(tiles_per_item), 1 if use_graph else 0)
        h = ctypes.c_void_p()
        _check(lib().ccq_batch_create(ctx.h, parr, n, rarr, ctypes.byref(opts), ctypes.byref(h)))
        self.h = h
        self._refresh_info()

    def _refresh_info(self):
        w, n = ctypes.c_size_t(), ctypes.c_int64()
        _check(lib().ccq_batch_info(self.h, ctypes.byref(w), ctypes.byref(n)))
        self.workspace_bytes, self.n_items = w.value, n.value

    def new_workspace(self):
        import torch
        return torch.empty(max(self.workspace_bytes, 256), dtype=torch.uint8, device="cuda:%d" % self.ctx.device)

    def set_tiles_per_item(self, t):
        _check(lib().ccq_batch_set_tiles_per_item(self.h, int(t)))
        self._refresh_info()

    def execute(self, workspace, stream=None, fused_events=None):
        """Enqueue the batch on `stream`.  fused_events: optional (begin, end)
        torch.cuda.Event pair recorded around the batch's persistent launches
        (such an execution is launched directly, not replayed from a graph)."""
        if fused_events is None:
            _check(lib().ccq_batch_execute(self.h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                           _stream_ptr(stream)))
            return
        opts = ExecOpts(_event_handle(fused_events[0], stream), _event_handle(fused_events[1], stream))
        _check(lib().ccq_batch_execute_ex(self.h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                          _stream_ptr(stream), ctypes.byref(opts)))

    def autotune(self, workspace, candidates=(8, 32, 128, 512), reps=3, stream=None):
        arr = (ctypes.c_int32 * len(candidates))(*candidates)
        best, ms = ctypes.c_int32(), ctypes.c_float()
        _check(lib().ccq_batch_autotune(self.h, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                                        _stream_ptr(stream), arr, len(candidates), int(reps), ctypes.byref(best),
                                        ctypes.byref(ms)))
        self._refresh_info()
        return best.value, ms.value

    def to_python(self):
        return [r.to_python() for r in self.results]

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ccq_batch_destroy(self.h)
            self.h = None


class Server:
    """Continuous-batching query server (ccq_server_*).  submit() returns a
    ticket; the plan and result stay referenced here until the ticket's
    completion has been polled."""

    def __init__(self, ctx, hbm_budget_bytes, max_inflight=64, max_batch=0, n_streams=2, batching=True,
                 tiles_per_item=0, graphs=True):
        self.ctx = ctx
        cfg = ServerConfig(int(hbm_budget_bytes), int(max_inflight), int(max_batch), int(n_streams),
                           1 if batching else 0, int(tiles_per_item), 0 if graphs else 1)
        h = ctypes.c_void_p()
        _check(lib().ccq_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._live = {}

    def submit(self, plan, result):
        t = ctypes.c_uint64()
        _check(lib().ccq_server_submit(self.h, plan.h, ctypes.byref(result.desc), ctypes.byref(t)))
        self._live[t.value] = (plan, result)
        return t.value

    def poll(self, max_n=1024):
        """Completed queries: list of dicts (ticket, status, t_submit, t_start, t_done)."""
        arr = (Completion * max_n)()
        n = ctypes.c_int32()
        _check(lib().ccq_server_poll(self.h, arr, max_n, ctypes.byref(n)))
        out = []
        for i in range(n.value):
            c = arr[i]
            self._live.pop(c.ticket, None)
            out.append({"ticket": c.ticket, "status": c.status, "t_submit": c.t_submit, "t_start": c.t_start,
                        "t_done": c.t_done})
        return out

    def drain(self, timeout_s=60.0):
        _check(lib().ccq_server_drain(self.h, float(timeout_s)))

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ccq_server_destroy(self.h)
            self.h = None
        self._live = {}

    def __del__(self):
        self.close()


def now():
    """The host steady clock the server stamps completions with (seconds)."""
    return lib().ccq_now()


def to_device(columns, device="cuda:0"):
    """Host column dicts (numpy) -> device column dicts (torch tensors)."""
    import torch
    out = {}
    for name, c in columns.items():
        d = {"enc": c["enc"]}
        for k, v in c.items():
            if isinstance(v, np.ndarray):
                if v.dtype == np.uint32:
                    v = v.view(np.int32)
                d[k] = torch.from_numpy(np.ascontiguousarray(v)).to(device)
            elif k != "enc":
                d[k] = v
        out[name] = d
    return out


# ---- encoding Plain data on the device (ccq_encode_*, ccq_plain_to_*)

def _enc_ws(values):
    import torch
    n = values.numel()
    return torch.empty(max(int(lib().ccq_encode_workspace_bytes(n)), 256), dtype=torch.uint8, device=values.device)


def encode_choose(ctx, values, stream=None):
    """Column statistics and the chosen encoding (dict) of a device tensor."""
    values = values.contiguous()
    ws = _enc_ws(values)
    out = EncodingChoice()
    _check(lib().ccq_encode_choose(ctx.h, ctypes.c_void_p(values.data_ptr()), _dtype_code(values), values.numel(),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream),
                                   ctypes.byref(out)))
    d = {k: getattr(out, k) for k, _ in EncodingChoice._fields_}
    d["choice"] = CHOICE_NAMES[d["choice"]]
    return d


def plain_to_rle(ctx, values, stream=None):
    """Device Plain -> RLE column dict (run values, exclusive run ends)."""
    import torch
    values = values.contiguous()
    ws = _enc_ws(values)
    n = ctypes.c_int64()
    L = lib()
    args = lambda rv, re_, cap: (ctx.h, ctypes.c_void_p(values.data_ptr()), _dtype_code(values), values.numel(),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), rv, re_, cap,
                                 ctypes.byref(n))
    st = L.ccq_plain_to_rle(*args(None, None, 0))
    if st != E_CAPACITY:
        _check(st)
    rv = torch.empty(max(n.value, 1), dtype=values.dtype, device=values.device)
    re_ = torch.empty(max(n.value, 1), dtype=torch.int64, device=values.device)
    _check(L.ccq_plain_to_rle(*args(ctypes.c_void_p(rv.data_ptr()), ctypes.c_void_p(re_.data_ptr()), n.value)))
    return {"enc": "rle", "values": rv[:n.value], "run_ends": re_[:n.value]}


def plain_to_rle_index(ctx, values, stream=None):
    """Device Plain -> RLE+Index: {"runs": {values, starts, ends}, "points": {positions, values}}."""
    import torch
    values = values.contiguous()
    ws = _enc_ws(values)
    nr, npt = ctypes.c_int64(), ctypes.c_int64()
    L = lib()
    dev = values.device

    def call(bufs, rc, pc):
        p = [ctypes.c_void_p(b.data_ptr()) if b is not None else None for b in bufs]
        return L.ccq_plain_to_rle_index(ctx.h, ctypes.c_void_p(values.data_ptr()), _dtype_code(values),
                                        values.numel(), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream_ptr(stream), p[0], p[1], p[2], rc, p[3], p[4], pc,
                                        ctypes.byref(nr), ctypes.byref(npt))
    st = call([None] * 5, 0, 0)
    if st != E_CAPACITY and st != OK:
        _check(st)
    r, q = nr.value, npt.value
    bufs = [torch.empty(max(r, 1), dtype=values.dtype, device=dev), torch.empty(max(r, 1), dtype=torch.int64, device=dev),
            torch.empty(max(r, 1), dtype=torch.int64, device=dev), torch.empty(max(q, 1), dtype=torch.int64, device=dev),
            torch.empty(max(q, 1), dtype=values.dtype, device=dev)]
    _check(call(bufs, r, q))
    return {"runs": {"values": bufs[0][:r], "starts": bufs[1][:r], "ends": bufs[2][:r]},
            "points": {"positions": bufs[3][:q], "values": bufs[4][:q]}}


def plain_to_plain_index(ctx, values, bit_width, base, stream=None):
    """Device Plain -> Plain+Index: a bit-packed column dict (codes value -
    base; rows outside [base, base + 2^w) hold 0) and the outliers as points."""
    import torch
    values = values.contiguous()
    ws = _enc_ws(values)
    n = values.numel()
    words = (n * int(bit_width) + 31) // 32 + 2
    packed = torch.empty(words, dtype=torch.int32, device=values.device)
    npt = ctypes.c_int64()
    L = lib()

    def call(pos, vals, cap):
        return L.ccq_plain_to_plain_index(ctx.h, ctypes.c_void_p(values.data_ptr()), _dtype_code(values), n,
                                          int(bit_width), int(base), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream_ptr(stream), ctypes.c_void_p(packed.data_ptr()), words,
                                          pos, vals, cap, ctypes.byref(npt))
    st = call(None, None, 0)
    if st != E_CAPACITY and st != OK:
        _check(st)
    q = npt.value
    pos = torch.empty(max(q, 1), dtype=torch.int64, device=values.device)
    vals = torch.empty(max(q, 1), dtype=values.dtype, device=values.device)
    _check(call(ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(vals.data_ptr()), q))
    return {"column": {"enc": "bitpacked", "packed": packed, "w": int(bit_width), "base": int(base)},
            "points": {"positions": pos[:q], "values": vals[:q]}}


# ---- joins (ccq_join_*)

def _col_index(table, col):
    return table.names.index(col) if isinstance(col, str) else int(col)


def join_index(left, left_col, right, right_col, left_window=None, right_window=None, stream=None):
    """Get Join Index of two tables' columns: (blocks, n_pairs), blocks an
    int64 device tensor [n, 4] of (left_start, left_len, right_start,
    right_len) rows."""
    import torch
    lw = left_window or (0, left.n_rows)
    rw = right_window or (0, right.n_rows)
    L = lib()
    lc, rc = _col_index(left, left_col), _col_index(right, right_col)
    wsb = L.ccq_join_workspace_bytes(left.h, lc, lw[0], lw[1], right.h, rc, rw[0], rw[1])
    if wsb == 0:          # the size call fails only on invalid arguments
        raise CcqError(E_INVALID, L.ccq_last_error().decode())
    dev = torch.device("cuda", left.ctx.device)
    ws = torch.empty(max(int(wsb), 256), dtype=torch.uint8, device=dev)
    nb, npairs = ctypes.c_int64(), ctypes.c_int64()

    def call(buf, cap):
        return L.ccq_join_index(left.h, lc, lw[0], lw[1], right.h, rc, rw[0], rw[1], ctypes.c_void_p(ws.data_ptr()),
                                ws.numel(), _stream_ptr(stream), buf, cap, ctypes.byref(nb), ctypes.byref(npairs))
    st = call(None, 0)
    if st != E_CAPACITY and st != OK:
        _check(st)
    blocks = torch.empty((max(nb.value, 1), 4), dtype=torch.int64, device=dev)
    if nb.value:
        _check(call(ctypes.c_void_p(blocks.data_ptr()), nb.value))
    return blocks[:nb.value], npairs.value


def join_apply(table, col, blocks, side, stream=None):
    """Apply Join Index: the column's values at the `side` ("left"/0 or
    "right"/1) rows of the blocks' pairs, an int64 device tensor."""
    import torch
    blocks = blocks.contiguous()
    sd = {"left": 0, "right": 1}.get(side, side)
    L = lib()
    n = blocks.shape[0]
    dev = torch.device("cuda", table.ctx.device)
    n_out = ctypes.c_int64()
    ci = _col_index(table, col)

    def call(ws, buf, cap):
        return L.ccq_join_apply(table.h, ci, ctypes.c_void_p(blocks.data_ptr()) if n else None, n, sd,
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream), buf, cap,
                                ctypes.byref(n_out))
    # first call: the number of pairs (the workspace grows with it)
    ws = torch.empty(max(int(L.ccq_join_apply_workspace_bytes(n, 0)), 256), dtype=torch.uint8, device=dev)
    st = call(ws, None, 0)
    if st != E_CAPACITY and st != OK:
        _check(st)
    total = n_out.value
    out = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
    if total:
        ws = torch.empty(max(int(L.ccq_join_apply_workspace_bytes(n, total)), 256), dtype=torch.uint8, device=dev)
        _check(call(ws, ctypes.c_void_p(out.data_ptr()), total))
    return out[:total]


def avg_var(count, s, ss):
    """AVG and VAR per result row from COUNT, SUM(x), SUM(x * x) (host
    lists or arrays of int64), through ccq_avg_var."""
    c = np.ascontiguousarray(np.asarray(count, dtype=np.int64))
    a = np.ascontiguousarray(np.asarray(s, dtype=np.int64))
    q = np.ascontiguousarray(np.asarray(ss, dtype=np.int64))
    avg, var = np.zeros(len(c)), np.zeros(len(c))
    _check(lib().ccq_avg_var(c.ctypes.data, a.ctypes.data, q.ctypes.data, len(c), avg.ctypes.data, var.ctypes.data))
    return avg.tolist(), var.tolist()

"""ctypes wrapper around the CPU oracle (``libccq_oracle.so``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the GPU library.  It converts the
column / query dicts described in ``datagen`` into the oracle's own structs.

Results are returned as plain Python values::

    {"keys": [tuple, ...], "counts": [int, ...], "aggs": [tuple, ...]}

in ascending key order; an ungrouped query returns exactly one row.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("CCQ_ORACLE_LIB") or os.path.join(_HERE, "libccq_oracle.so")
_lib = None

RLE, INDEX, BITPACKED, RLE_INDEX, PLAIN_INDEX = 1, 2, 3, 4, 5
I32, I64 = 1, 2
RANGE, IN, NOT_RANGE, NOT_IN = 1, 2, 3, 4
COUNT, SUM, MIN, MAX = 1, 2, 3, 4
OPS = {"+": 1, "-": 2, "*": 3}


class OrcColumn(ctypes.Structure):
    _fields_ = [("enc", ctypes.c_int32), ("vtype", ctypes.c_int32), ("n", ctypes.c_int64),
                ("values", ctypes.c_void_p), ("run_ends", ctypes.c_void_p), ("positions", ctypes.c_void_p),
                ("packed", ctypes.c_void_p), ("w", ctypes.c_int32), ("ptype", ctypes.c_int32),
                ("base", ctypes.c_int64), ("run_starts", ctypes.c_void_p), ("pt_n", ctypes.c_int64),
                ("pt_positions", ctypes.c_void_p), ("pt_values", ctypes.c_void_p), ("pt_ptype", ctypes.c_int32),
                ("pt_vtype", ctypes.c_int32)]


class OrcPred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("op", ctypes.c_int32), ("lo", ctypes.c_int64), ("hi", ctypes.c_int64),
                ("in_list", ctypes.c_void_p), ("in_len", ctypes.c_int64), ("clause", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]


class OrcKey(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("shift", ctypes.c_int32), ("card", ctypes.c_int64)]


class OrcAgg(ctypes.Structure):
    _fields_ = [("func", ctypes.c_int32), ("col", ctypes.c_int32), ("op", ctypes.c_int32), ("col2", ctypes.c_int32)]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ -O2 (no SIMD intrinsics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               os.path.join(_HERE, "ccq_oracle.cpp"), "-o", tmp, "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_query.restype = ctypes.c_void_p
        L.orc_query.argtypes = [ctypes.POINTER(OrcColumn), ctypes.c_int32, ctypes.c_int64,
                                ctypes.POINTER(OrcPred), ctypes.c_int32, ctypes.POINTER(OrcKey), ctypes.c_int32,
                                ctypes.POINTER(OrcAgg), ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_int32]
        L.orc_error.restype = ctypes.c_char_p
        L.orc_error.argtypes = [ctypes.c_void_p]
        L.orc_n_groups.restype = ctypes.c_int64
        L.orc_n_groups.argtypes = [ctypes.c_void_p]
        L.orc_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_free.argtypes = [ctypes.c_void_p]
        L.orc_decode.restype = ctypes.c_char_p
        L.orc_decode.argtypes = [ctypes.POINTER(OrcColumn), ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_void_p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _vtype(a):
    if a.dtype == np.int32:
        return I32
    if a.dtype == np.int64:
        return I64
    raise OracleError("values must be int32 or int64, got %s" % a.dtype)


def _column(c, n_rows, keep):
    """Build an OrcColumn; `keep` holds the arrays alive."""
    oc = OrcColumn()
    if c["enc"] == "rle":
        v = np.ascontiguousarray(c["values"])
        e = np.ascontiguousarray(c["run_ends"], dtype=np.int64)
        if len(v) != len(e):
            raise OracleError("RLE values and run_ends differ in length")
        keep += [v, e]
        oc.enc, oc.vtype, oc.n = RLE, _vtype(v), len(e)
        oc.values, oc.run_ends = v.ctypes.data, e.ctypes.data
    elif c["enc"] == "index":
        v = np.ascontiguousarray(c["values"])
        p = np.ascontiguousarray(c["positions"])
        if len(v) != len(p):
            raise OracleError("Index values and positions differ in length")
        keep += [v, p]
        oc.enc, oc.vtype, oc.n, oc.ptype = INDEX, _vtype(v), len(p), _vtype(p)
        oc.values, oc.positions = v.ctypes.data, p.ctypes.data
    elif c["enc"] in ("bitpacked", "plain+index"):
        pk = np.ascontiguousarray(c["packed"], dtype=np.uint32)
        w = int(c["w"])
        if len(pk) < (n_rows * w + 31) // 32 + 2:
            raise OracleError("packed stream shorter than ceil(rows*w/32) + 2 words")
        keep.append(pk)
        oc.enc, oc.n, oc.w, oc.base = BITPACKED, n_rows, w, int(c.get("base", 0))
        oc.packed = pk.ctypes.data
        if c["enc"] == "plain+index":
            oc.enc = PLAIN_INDEX
            _points(oc, c, keep)
    elif c["enc"] == "rle+index":
        # Section 3.2 form: pure runs (values, starts, exclusive ends) and
        # points on the remaining rows
        v = np.ascontiguousarray(c["values"])
        s0 = np.ascontiguousarray(c["run_starts"], dtype=np.int64)
        e = np.ascontiguousarray(c["run_ends"], dtype=np.int64)
        if not len(v) == len(s0) == len(e):
            raise OracleError("RLE part values, run_starts and run_ends differ in length")
        keep += [v, s0, e]
        oc.enc, oc.vtype, oc.n = RLE_INDEX, _vtype(v), len(e)
        oc.values, oc.run_starts, oc.run_ends = v.ctypes.data, s0.ctypes.data, e.ctypes.data
        _points(oc, c, keep)
    else:
        raise OracleError("unknown encoding %r" % (c["enc"],))
    return oc


def _points(oc, c, keep):
    """The Index part of a composite column (positions, point_values)."""
    p = np.ascontiguousarray(c["positions"])
    v = np.ascontiguousarray(c["point_values"])
    if len(p) != len(v):
        raise OracleError("point positions and values differ in length")
    keep += [p, v]
    oc.pt_n, oc.pt_ptype, oc.pt_vtype = len(p), _vtype(p), _vtype(v)
    oc.pt_positions, oc.pt_values = p.ctypes.data, v.ctypes.data


def decode(column, n_rows, r0=0, r1=None):
    """Decompress rows [r0, r1) of one column to int64 (the oracle's decoder)."""
    r1 = n_rows if r1 is None else r1
    keep = []
    oc = _column(column, n_rows, keep)
    out = np.empty(max(r1 - r0, 0), dtype=np.int64)
    err = lib().orc_decode(ctypes.byref(oc), int(n_rows), int(r0), int(r1), out.ctypes.data)
    if err:
        raise OracleError(err.decode())
    return out


def run(table, query, n_threads=None):
    """Execute `query` over `table` ({"n_rows", "columns"}) on the CPU."""
    n_rows = int(table["n_rows"])
    names = list(table["columns"].keys())
    idx = {n: i for i, n in enumerate(names)}
    keep = []
    cols = (OrcColumn * max(len(names), 1))()
    for i, n in enumerate(names):
        cols[i] = _column(table["columns"][n], n_rows, keep)

    def col_id(name):
        if name not in idx:
            raise OracleError("unknown column %r" % (name,))
        return idx[name]

    # the filter: every entry of "preds" AND every clause of "or", a clause
    # being the OR of its predicates (Section 5.2)
    flat = [(p, 0) for p in query["preds"]]
    for k, clause in enumerate(query.get("or", ())):
        if not clause:
            raise OracleError("empty OR clause")
        flat += [(p, k + 1) for p in clause]
    preds = (OrcPred * max(len(flat), 1))()
    for i, (p, clause) in enumerate(flat):
        op = p[1]
        preds[i].col = col_id(p[0])
        preds[i].clause = clause
        if op in ("range", "not_range"):
            preds[i].op = RANGE if op == "range" else NOT_RANGE
            preds[i].lo, preds[i].hi = int(p[2]), int(p[3])
        elif op in ("in", "not_in"):
            lst = np.ascontiguousarray(np.array(list(p[2]), dtype=np.int64))
            keep.append(lst)
            preds[i].op = IN if op == "in" else NOT_IN
            preds[i].in_list, preds[i].in_len = lst.ctypes.data, len(lst)
        else:
            raise OracleError("unknown predicate %r" % (op,))
    keys = (OrcKey * max(len(query["keys"]), 1))()
    dicts = []
    for i, k in enumerate(query["keys"]):
        keys[i].col, keys[i].shift, keys[i].card = col_id(k[0]), int(k[1]), int(k[2])
        d = table["columns"][k[0]].get("dict")
        if d is not None:
            d = np.asarray(d, dtype=np.int64)
            if int(k[1]) != 0 or int(k[2]) > len(d):
                raise OracleError("a key on a dictionary column needs shift 0 and card <= the dictionary size")
        dicts.append(d)
    for a in query["aggs"]:
        if a[0] in ("sum", "min", "max"):
            args = a[1] if isinstance(a[1], tuple) else (a[1],)
            if any(table["columns"].get(c, {}).get("dict") is not None for c in args[::2]):
                raise OracleError("aggregate over a dictionary-encoded column")
    aggs = (OrcAgg * max(len(query["aggs"]), 1))()
    for i, a in enumerate(query["aggs"]):
        if a[0] == "count":
            aggs[i].func, aggs[i].col = COUNT, -1
        elif a[0] in ("sum", "min", "max"):
            aggs[i].func = {"sum": SUM, "min": MIN, "max": MAX}[a[0]]
            if isinstance(a[1], tuple):        # (col, op, col2): the row-wise col op col2
                c1, op, c2 = a[1]
                if op not in OPS:
                    raise OracleError("unknown operator %r" % (op,))
                aggs[i].col, aggs[i].op, aggs[i].col2 = col_id(c1), OPS[op], col_id(c2)
            else:
                aggs[i].col = col_id(a[1])
        else:
            raise OracleError("unknown aggregate %r" % (a[0],))
    rb, re_ = query.get("window", (0, n_rows))
    if n_threads is None:
        n_threads = os.cpu_count() or 1
    L = lib()
    h = L.orc_query(cols, len(names), n_rows, preds, len(flat), keys, len(query["keys"]), aggs,
                    len(query["aggs"]), int(rb), int(re_), int(n_threads))
    try:
        err = L.orc_error(h)
        if err:
            raise OracleError(err.decode())
        g = L.orc_n_groups(h)
        nk, na = len(query["keys"]), len(query["aggs"])
        kb = np.zeros(max(g * nk, 1), dtype=np.int64)
        cb = np.zeros(max(g, 1), dtype=np.int64)
        ab = np.zeros(max(g * na, 1), dtype=np.int64)
        L.orc_copy(h, kb.ctypes.data, cb.ctypes.data, ab.ctypes.data)
    finally:
        L.orc_free(h)
    # Dictionary encoding (Section 2.1) stores a code per row and the
    # distinct values once: a key on such a column is a code, and the result
    # reports the value the code stands for, dict[code].  Groups keep the
    # order of their codes.
    def decode(j, x):
        return int(x) if dicts[j] is None else int(dicts[j][int(x)])

    return {
        "keys": [tuple(decode(j, x) for j, x in enumerate(kb[i * nk:(i + 1) * nk])) for i in range(g)],
        "counts": [int(x) for x in cb[:g]],
        "aggs": [tuple(int(x) for x in ab[i * na:(i + 1) * na]) for i in range(g)],
    }


# ---- NOT on position-explicit masks (Section 5.3; Appendix, NOT operator)
#
# A mask in RLE form lists inclusive row ranges [start_i, end_i] (sorted,
# disjoint); in Index form it lists single rows.  The complement of an RLE
# mask is the list of gaps between its ranges (Algorithm 7), that of an
# Index mask the gaps between its rows, also as ranges (Algorithm 8).  These
# are the paper's mask forms, kept here to pin the meaning of NOT that the
# query path evaluates per row.

def not_rle(start, end, total_size):
    """Gaps of an RLE mask over rows [0, total_size): each candidate gap runs
    from one range's end + 1 to the next range's start - 1; empty ones drop."""
    s2 = [e + 1 for e in [-1] + list(end)]
    e2 = [s - 1 for s in list(start) + [total_size]]
    keep = [i for i in range(len(s2)) if s2[i] <= e2[i]]
    return [s2[i] for i in keep], [e2[i] for i in keep]


def not_index(pos, total_size):
    """Gaps of an Index mask over rows [0, total_size), as RLE ranges."""
    s2 = [p + 1 for p in [-1] + list(pos)]
    e2 = [p - 1 for p in list(pos) + [total_size]]
    keep = [i for i in range(len(s2)) if s2[i] <= e2[i] and s2[i] < total_size and e2[i] >= 0]
    return [s2[i] for i in keep], [e2[i] for i in keep]


# ---- OR on position-explicit masks (Section 5.2; Tables 4 and 5)
#
# The OR of two Plain masks is the element-wise OR; that of two RLE masks is
# the union of their row ranges, as maximal ranges of consecutive passing
# rows; that of two Index masks is the sorted union of their rows.  The query
# path evaluates OR per row; these pin what that means on the paper's masks.

def or_plain(m1, m2):
    """Element-wise OR of two boolean masks of one length."""
    if len(m1) != len(m2):
        raise OracleError("masks of different lengths")
    return [bool(a) or bool(b) for a, b in zip(m1, m2)]


def range_union(start1, end1, start2, end2):
    """Union of two RLE masks (sorted, disjoint inclusive ranges each): the
    ranges of both, taken by start, with each range that overlaps or touches
    the one before folded into it."""
    ranges = sorted(zip(list(start1) + list(start2), list(end1) + list(end2)))
    s_out, e_out = [], []
    for s, e in ranges:
        if e_out and s <= e_out[-1] + 1:
            e_out[-1] = max(e_out[-1], e)
        else:
            s_out.append(s)
            e_out.append(e)
    return s_out, e_out


def merge_sorted_idx(pos1, pos2):
    """Union of two Index masks (sorted, unique rows each), sorted, each row
    once: a two-way merge."""
    out = []
    i = j = 0
    while i < len(pos1) or j < len(pos2):
        if j == len(pos2) or (i < len(pos1) and pos1[i] <= pos2[j]):
            x = pos1[i]
            i += 1
        else:
            x = pos2[j]
            j += 1
        if not out or out[-1] != x:
            out.append(x)
    return out


def concat_sort(pos1, pos2):
    """Union of two Index masks for small inputs: both lists joined, sorted,
    repeated rows dropped."""
    return sorted(set(int(x) for x in list(pos1) + list(pos2)))


# ---- AND of two Index masks (Algorithm 4, idx_in_idx)

def idx_in_idx(pos1, pos2):
    """Rows of Index mask pos1 also in Index mask pos2 (both sorted, unique):
    for each row of pos1, the last row of pos2 at or before it (an upper-bound
    bucketize, minus one) must be that row itself."""
    pos1 = np.asarray(pos1, dtype=np.int64)
    pos2 = np.asarray(pos2, dtype=np.int64)
    b = np.searchsorted(pos2, pos1, side="right") - 1
    ok = b >= 0
    ok[ok] = pos2[b[ok]] == pos1[ok]
    return [int(x) for x in pos1[ok]]


# ---- AVG and VAR as post-processing of SUM and COUNT (Section 7.2,
# aggregating phase: AVG divides SUM by COUNT; STD and VAR need the sum of
# the squared values too).  The exact integer aggregates are rounded to the
# nearest double each, then combined in IEEE double arithmetic in this
# order (population variance): avg = s / n; var = (ss - s * s / n) / n.
# A group with n = 0 (the empty ungrouped row) gives 0.0 for both.

def avg_var(count, s, ss):
    n, s_, ss_ = float(count), float(s), float(ss)
    if count == 0:
        return 0.0, 0.0
    return s_ / n, (ss_ - s_ * s_ / n) / n

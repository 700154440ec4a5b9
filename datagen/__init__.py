"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

This module only *produces* encoded columns and query descriptions; it holds
none of the query arithmetic (no predicate evaluation, alignment, grouping or
aggregation).  Both the oracle and the GPU library consume exactly the bytes
made here.

Column dicts (plain numpy arrays, host memory):

* RLE:        {"enc": "rle", "values": int32|int64[R], "run_ends": int64[R]}
              run_ends are exclusive, strictly increasing, last == n_rows.
* Index:      {"enc": "index", "positions": int32[nnz], "values": int32|int64[nnz]}
              positions strictly increasing in [0, n_rows); unlisted rows hold 0.
* Bit-packed: {"enc": "bitpacked", "packed": uint32[W], "w": w, "base": b}
              row r holds base + bits [r*w, r*w + w) of the LSB-first stream.

A query dict:

    {"preds":  [(col, "range", lo, hi) | (col, "in", [v, ...]), ...],   # AND
     "keys":   [(col, shift, card), ...],      # key = value >> shift in [0, card)
     "aggs":   [("count",) | ("sum", col), ...],
     "window": (row_begin, row_end)}
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libccq_datagen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the generator library with gcc (OpenMP, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        src = os.path.join(_HERE, "dg.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", src,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        u64, i64, dbl, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_int
        vp = ctypes.c_void_p
        L.dg_rle_count.restype = i64
        L.dg_rle_count.argtypes = [u64, u64, i32, dbl, dbl, i64]
        L.dg_rle_fill.restype = None
        L.dg_rle_fill.argtypes = [u64, u64, i32, dbl, dbl, i64, vp, i64]
        L.dg_uniform_i32.argtypes = [u64, u64, i64, i64, vp, i64]
        L.dg_uniform_i64.argtypes = [u64, u64, i64, i64, vp, i64]
        L.dg_sparse_count.restype = i64
        L.dg_sparse_count.argtypes = [u64, u64, dbl, i64]
        L.dg_sparse_fill.argtypes = [u64, u64, dbl, i64, vp, i64]
        L.dg_sparse_fill64.argtypes = [u64, u64, dbl, i64, vp, i64]
        L.dg_zipf_codes.argtypes = [u64, u64, dbl, i64, vp, i64]
        L.dg_zipf_pmf.argtypes = [dbl, i64, vp]
        L.dg_packed_words.restype = i64
        L.dg_packed_words.argtypes = [i64, i32]
        L.dg_pack.argtypes = [vp, i64, i32, vp, i64]
        L.dg_codes_packed.argtypes = [u64, u64, i32, dbl, i64, i64, i32, vp, i64]
        L.dg_max_threads.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------- primitives

def rle_column(seed, stream, n_rows, dist, mean, vlo, vhi, vdtype=np.int32, sigma=1.0):
    """RLE column: run lengths geometric ("geometric", mean) or lognormal
    ("lognormal", mean, sigma), i.i.d. values uniform in [vlo, vhi)."""
    L = lib()
    d = {"geometric": 0, "lognormal": 1}[dist]
    R = L.dg_rle_count(seed, stream, d, float(mean), float(sigma), int(n_rows))
    ends = np.empty(R, dtype=np.int64)
    L.dg_rle_fill(seed, stream, d, float(mean), float(sigma), int(n_rows), _ptr(ends), R)
    vals = np.empty(R, dtype=vdtype)
    if vdtype == np.int32:
        L.dg_uniform_i32(seed, stream + 1, int(vlo), int(vhi), _ptr(vals), R)
    else:
        L.dg_uniform_i64(seed, stream + 1, int(vlo), int(vhi), _ptr(vals), R)
    return {"enc": "rle", "values": vals, "run_ends": ends}


def sparse_column(seed, stream, n_rows, density, vlo, vhi, vdtype=np.int64):
    """Index column: each row listed independently with probability `density`,
    values uniform in [vlo, vhi); int32 positions, int64 past 2^31 rows."""
    L = lib()
    n = L.dg_sparse_count(seed, stream, float(density), int(n_rows))
    if n_rows <= (1 << 31) - 1:
        pos = np.empty(n, dtype=np.int32)
        L.dg_sparse_fill(seed, stream, float(density), int(n_rows), _ptr(pos), n)
    else:
        # positions past 2^31: int64 (the same rows as the int32 form would list)
        pos = np.empty(n, dtype=np.int64)
        L.dg_sparse_fill64(seed, stream, float(density), int(n_rows), _ptr(pos), n)
    vals = np.empty(n, dtype=vdtype)
    if vdtype == np.int32:
        L.dg_uniform_i32(seed, stream + 1, int(vlo), int(vhi), _ptr(vals), n)
    else:
        L.dg_uniform_i64(seed, stream + 1, int(vlo), int(vhi), _ptr(vals), n)
    return {"enc": "index", "positions": pos, "values": vals}


def packed_words(n, w):
    return int(lib().dg_packed_words(int(n), int(w)))


def pack_codes(codes, w):
    """Pack uint32 codes (low w bits each) into the LSB-first stream."""
    codes = np.ascontiguousarray(codes, dtype=np.uint32)
    nw = packed_words(len(codes), w)
    out = np.empty(nw, dtype=np.uint32)
    lib().dg_pack(_ptr(codes), len(codes), int(w), _ptr(out), nw)
    return out


def zipf_codes(seed, stream, s, n_codes, n):
    out = np.empty(n, dtype=np.uint32)
    lib().dg_zipf_codes(seed, stream, float(s), int(n_codes), _ptr(out), int(n))
    return out


def zipf_pmf(s, n_codes):
    out = np.empty(n_codes, dtype=np.float64)
    lib().dg_zipf_pmf(float(s), int(n_codes), _ptr(out))
    return out


def packed_column(seed, stream, n_rows, w, kind, n_codes, s=1.1, base=0):
    """Bit-packed column of codes drawn Zipf(s) ("zipf") or uniform ("uniform")
    over [0, n_codes), value = base + code."""
    nw = packed_words(n_rows, w)
    out = np.empty(nw, dtype=np.uint32)
    k = {"zipf": 0, "uniform": 1}[kind]
    lib().dg_codes_packed(seed, stream, k, float(s), int(n_codes), int(n_rows), int(w), _ptr(out), nw)
    return {"enc": "bitpacked", "packed": out, "w": int(w), "base": int(base)}


def in_list_by_weight(seed, pmf, k):
    """k distinct codes drawn with probability proportional to pmf, sorted."""
    rng = np.random.default_rng([int(seed), 999])
    pick = rng.choice(len(pmf), size=k, replace=False, p=pmf / pmf.sum())
    return sorted(int(x) for x in pick)


# ---------------------------------------------------------------- workloads

def config_c1(seed=1, n_rows=1_000_000):
    """Two RLE int32 columns over n_rows rows: a (geometric runs, mean 16) and
    b (geometric runs, mean 40), values uniform in [0, 1000);
    SELECT SUM(b), COUNT(*) WHERE a < 500."""
    cols = {
        "a": rle_column(seed, 1010, n_rows, "geometric", 16, 0, 1000),
        "b": rle_column(seed, 1020, n_rows, "geometric", 40, 0, 1000),
    }
    q = {"preds": [("a", "range", -(1 << 63), 500)], "keys": [],
         "aggs": [("sum", "b"), ("count",)], "window": (0, n_rows)}
    return {"name": "c1_two_rle_1e6", "n_rows": n_rows, "columns": cols, "query": q}


C2_COLS = ("r0", "r1", "r2", "s", "d", "p")


def config_c2(seed=2, n_rows=1_000_000_000, columns=("r0", "r1", "s", "d")):
    """Mixed encodings over n_rows rows:
    r0, r1, r2 RLE int32 (lognormal runs, sigma 1, means 64/200/1000, values
    uniform [0, 2^16)); s index-encoded int64 (1% of rows, values uniform
    [1, 1e6)); d dictionary codes (Zipf s=1.1 over 10k entries) packed to 14
    bits; p plain int32 packed to 20 bits around base -2^19.
    Query: r0 in [0,32768) AND r1 in [16384,65536) AND d IN (50 codes drawn by
    Zipf weight) GROUP BY d -> SUM(s), COUNT(*).  Only `columns` are built."""
    gen = {
        "r0": lambda: rle_column(seed, 2010, n_rows, "lognormal", 64, 0, 1 << 16),
        "r1": lambda: rle_column(seed, 2020, n_rows, "lognormal", 200, 0, 1 << 16),
        "r2": lambda: rle_column(seed, 2030, n_rows, "lognormal", 1000, 0, 1 << 16),
        "s": lambda: sparse_column(seed, 2040, n_rows, 0.01, 1, 1_000_000),
        "d": lambda: packed_column(seed, 2050, n_rows, 14, "zipf", 10000, s=1.1),
        "p": lambda: packed_column(seed, 2060, n_rows, 20, "uniform", 1 << 20, base=-(1 << 19)),
    }
    cols = {c: gen[c]() for c in columns}
    in_codes = in_list_by_weight(seed, zipf_pmf(1.1, 10000), 50)
    q = {"preds": [("r0", "range", 0, 32768), ("r1", "range", 16384, 65536), ("d", "in", in_codes)],
         "keys": [("d", 0, 10000)],
         "aggs": [("sum", "s"), ("count",)], "window": (0, n_rows)}
    return {"name": "c2_mixed_%g" % n_rows, "n_rows": n_rows, "columns": cols, "query": q}


def config_c3(seed=3, n_rows=10_000_000_000):
    """Four RLE int32 key columns (lognormal runs, mean 256, values uniform in
    [0,100), [0,100), [0,10), [0,10)) and one RLE int64 measure (lognormal
    runs, mean 32, values uniform in [-1e6, 1e6]);
    GROUP BY k0, k1, k2, k3 -> SUM(m), COUNT(*)."""
    cards = (100, 100, 10, 10)
    cols = {}
    for i, c in enumerate(cards):
        cols["k%d" % i] = rle_column(seed, 3010 + 10 * i, n_rows, "lognormal", 256, 0, c)
    cols["m"] = rle_column(seed, 3060, n_rows, "lognormal", 32, -1_000_000, 1_000_001, np.int64)
    q = {"preds": [], "keys": [("k%d" % i, 0, c) for i, c in enumerate(cards)],
         "aggs": [("sum", "m"), ("count",)], "window": (0, n_rows)}
    return {"name": "c3_multi_rle_%g" % n_rows, "n_rows": n_rows, "columns": cols, "query": q}


def c4_queries(seed, n_rows, n_queries=4096, lo_rows=10_000, hi_rows=100_000_000):
    """Query templates over a table with config_c2's columns (r0, r1, r2, s,
    d, p): window length log-uniform in [lo_rows, hi_rows] (clipped to the
    table) at a uniform offset; 1-3 predicates drawn from {range on r0, r1,
    r2; IN on d with 1-50 codes; range on p}; 1-2 aggregates from {COUNT(*),
    SUM(s), SUM(r2), SUM(p)}; GROUP BY none, d, or r_j >> shift (1 to 10k
    groups)."""
    rng = np.random.default_rng([int(seed), 4444])
    pmf = zipf_pmf(1.1, 10000)
    out = []
    for _ in range(n_queries):
        n = int(round(10 ** rng.uniform(np.log10(lo_rows), np.log10(hi_rows))))
        n = max(1, min(n, n_rows))
        off = int(rng.integers(0, n_rows - n + 1))
        kinds = rng.choice(5, size=int(rng.integers(1, 4)), replace=False)
        preds = []
        for k in kinds:
            if k < 3:
                lo = int(rng.integers(0, 1 << 16))
                hi = lo + int(rng.integers(1 << 13, 1 << 16))
                preds.append(("r%d" % k, "range", lo, hi))
            elif k == 3:
                m = int(rng.integers(1, 51))
                codes = rng.choice(10000, size=m, replace=False, p=pmf)
                preds.append(("d", "in", sorted(int(c) for c in codes)))
            else:
                lo = int(rng.integers(-(1 << 19), 1 << 19))
                preds.append(("p", "range", lo, lo + int(rng.integers(1 << 16, 1 << 20))))
        aggs = [("count",), ("sum", "s"), ("sum", "r2"), ("sum", "p")]
        pick = rng.choice(4, size=int(rng.integers(1, 3)), replace=False)
        aggs = [aggs[i] for i in sorted(pick)]
        g = int(rng.integers(0, 3))
        if g == 0:
            keys = []
        elif g == 1:
            keys = [("d", 0, 10000)]
        else:
            shift = int(rng.integers(3, 17))
            keys = [("r%d" % int(rng.integers(0, 3)), shift, 1 << (16 - shift))]
        out.append({"preds": preds, "keys": keys, "aggs": aggs, "window": (off, off + n)})
    return out


def config_c4(seed=4, n_rows=100_000_000, n_queries=4096):
    """A table with config_c2's column mix over n_rows rows and n_queries
    query templates (see c4_queries)."""
    t = config_c2(seed=seed, n_rows=n_rows, columns=("r0", "r1", "r2", "s", "d", "p"))
    t["name"] = "c4_batch_%d_over_%g" % (n_queries, n_rows)
    t["queries"] = c4_queries(seed, n_rows, n_queries)
    return t

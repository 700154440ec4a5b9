"""CPU oracle for encoding Plain data (TEST INFRASTRUCTURE ONLY: imported by
the tests, never by the GPU library).

Plain definitions, written from the paper:
- plain_to_rle: Section 3.1 (RLE keeps a value per run of equal adjacent
  values with the run's start and end); we keep exclusive ends.
- plain_to_rle_index, plain_to_plain_index: Section 3.2 (composite
  encodings: single-row "impure" stretches as Index points beside RLE runs;
  outliers as Index points beside narrow Plain codes).
- choose: the evaluation setup's encoding heuristics (Section 9), with the
  readings spelled out in `choose`'s docstring.

The packer here is this module's own (numpy bit arrays), not the
generator's, so a bit-layout mistake on either side shows.
"""
from __future__ import annotations

import numpy as np

MIN_ROWS = 1_000_000      # columns under this many rows stay Plain
RATIO = 20.0              # compression ratio above which RLE (or RLE+Index) is chosen


def plain_to_rle(x):
    """Maximal runs: (run values, exclusive run ends)."""
    x = np.asarray(x)
    n = len(x)
    if n == 0:
        return x[:0].copy(), np.zeros(0, dtype=np.int64)
    starts = np.flatnonzero(np.concatenate([[True], x[1:] != x[:-1]]))
    ends = np.concatenate([starts[1:], [n]]).astype(np.int64)
    return x[starts].copy(), ends


def plain_to_rle_index(x):
    """Runs of two or more rows as RLE (values, starts, exclusive ends) and
    the rows that form a run alone as Index (positions, values)."""
    x = np.asarray(x)
    vals, ends = plain_to_rle(x)
    starts = np.concatenate([[0], ends[:-1]]).astype(np.int64) if len(ends) else np.zeros(0, dtype=np.int64)
    single = (ends - starts) == 1
    return ((vals[~single].copy(), starts[~single].copy(), ends[~single].copy()),
            (starts[single].copy(), vals[single].copy()))


def pack_bits(codes, w):
    """LSB-first stream of w-bit codes in little-endian uint32 words, row r at
    bits [r w, r w + w), plus two zero pad words."""
    codes = np.asarray(codes, dtype=np.uint64)
    n = len(codes)
    n_words = (n * w + 31) // 32 + 2
    bits = ((codes[:, None] >> np.arange(w, dtype=np.uint64)[None, :]) & np.uint64(1)).astype(np.uint8).ravel()
    bits = np.concatenate([bits, np.zeros(n_words * 32 - len(bits), dtype=np.uint8)])
    return np.packbits(bits, bitorder="little").view("<u4").astype(np.uint32)


def plain_to_plain_index(x, w, base):
    """Codes value - base where that lies in [0, 2^w), else 0 (the row is an
    outlier), packed; and the outliers as Index points."""
    x = np.asarray(x)
    xi = x.astype(np.int64)
    # value - base for the values >= base, exact in uint64 arithmetic
    d = xi.view(np.uint64) - np.array([int(base)], dtype=np.int64).view(np.uint64)[0]
    inside = (xi >= int(base)) & (d < np.uint64(1 << int(w)))
    codes = np.where(inside, d, np.uint64(0))
    pos = np.flatnonzero(~inside).astype(np.int64)
    return pack_bits(codes, int(w)), (pos, x[pos].copy())


def bits_for(span):
    """Fewest bits w >= 1 with span < 2^w (span >= 0)."""
    return max(1, int(span).bit_length())


def choose(x):
    """Column statistics and the encoding the Section 9 heuristics pick.

    Readings: the compression ratio is Plain bytes over the bytes of the
    paper's run representation, three elements per run (value, start, end:
    sizeof(value) + 16 bytes); RLE+Index is taken when single-row runs exist
    and the rows of the longer runs, over those runs' bytes, still compress
    by more than 20 (the single rows go to the Index part); the 5% cut keeps
    the values between sorted ranks floor(n/20) and n - 1 - floor(n/20); a
    "narrower type" is a smaller bit width; Plain with a range wider than 32
    bits (no bit-packed form) falls back to RLE."""
    x = np.asarray(x)
    n = len(x)
    out = {"n_rows": n, "runs": 0, "single_runs": 0, "min_value": 0, "max_value": 0, "lo_cut": 0, "hi_cut": 0,
           "choice": "plain", "bit_width": 0, "base": 0, "rle_runs": 0, "index_points": 0}
    if n == 0:
        out["bit_width"] = 1
        return out
    vals, ends = plain_to_rle(x)
    lengths = np.diff(np.concatenate([[0], ends]))
    out["runs"] = int(len(vals))
    out["single_runs"] = int((lengths == 1).sum())
    xs = np.sort(x.astype(np.int64))
    out["min_value"], out["max_value"] = int(xs[0]), int(xs[-1])
    out["lo_cut"], out["hi_cut"] = int(xs[n // 20]), int(xs[n - 1 - n // 20])
    vb = 4.0 if x.dtype == np.int32 else 8.0
    plain_bytes = n * vb
    longs = out["runs"] - out["single_runs"]
    w_full = bits_for(out["max_value"] - out["min_value"])
    w_cut = bits_for(out["hi_cut"] - out["lo_cut"])
    if n >= MIN_ROWS and plain_bytes / (out["runs"] * (vb + 16.0)) > RATIO:
        out.update(choice="rle", rle_runs=out["runs"])
    elif (n >= MIN_ROWS and out["single_runs"] > 0 and longs > 0 and
          (n - out["single_runs"]) * vb / (longs * (vb + 16.0)) > RATIO):
        out.update(choice="rle+index", rle_runs=longs, index_points=out["single_runs"])
    elif n >= MIN_ROWS and w_cut < w_full and w_cut <= 32:
        # centering: codes around the cut range's midpoint (rounded up), so
        # [lo_cut, hi_cut] lies inside [base, base + 2^w)
        span = out["hi_cut"] - out["lo_cut"]
        base = max(out["lo_cut"] + (span + 1) // 2 - (1 << (w_cut - 1)), -(1 << 63))
        xi = x.astype(np.int64)
        # value - base for the values >= base, exact in uint64 arithmetic
        d = xi.view(np.uint64) - np.array([base], dtype=np.int64).view(np.uint64)[0]
        outside = (xi < base) | (d >= np.uint64(1 << w_cut))
        out.update(choice="plain+index", bit_width=w_cut, base=base, index_points=int(outside.sum()))
    elif w_full <= 32:
        out.update(choice="plain", bit_width=w_full, base=out["min_value"])
    else:
        out.update(choice="rle", rle_runs=out["runs"])
    return out


def decode_rle(vals, ends):
    lengths = np.diff(np.concatenate([[0], np.asarray(ends, dtype=np.int64)]))
    return np.repeat(np.asarray(vals), lengths)


def decode_rle_index(runs, points, n, dtype):
    out = np.zeros(n, dtype=dtype)
    vals, starts, ends = runs
    for v, s, e in zip(vals, starts, ends):
        out[s:e] = v
    pos, pv = points
    out[np.asarray(pos, dtype=np.int64)] = pv
    return out


def decode_plain_index(packed, w, base, points, n, dtype):
    words = np.asarray(packed, dtype=np.uint32)
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")
    out = np.zeros(n, dtype=object)
    for r in range(n):
        code = 0
        for b in range(w):
            code |= int(bits[r * w + b]) << b
        out[r] = int(base) + code
    pos, pv = points
    for p, v in zip(pos, pv):
        out[int(p)] = int(v)
    return out.astype(dtype)

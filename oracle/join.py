"""CPU oracle for joins on encoded columns (TEST INFRASTRUCTURE ONLY:
imported by the tests, never by the GPU library).

Section 8 joins two columns in two steps.  Get Join Index finds every pair
of rows (one from each column) whose values are equal; Apply Join Index then
reads a column at the rows of one side, pair by pair.  The pairs are the
plain definition; the encodings only compress them:

- a join entry is a run of an RLE column (its value and row range, clipped
  to the window), a listed point of an Index column (its value at its
  position; unlisted rows are not rows of the joined relation: the join
  hashes the value tensor), or one row of a bit-packed column;
- two entries with equal values give one *block*: the cross product of the
  left entry's rows and the right entry's rows (Table 6: an RLE side keeps
  its join index as row ranges, the other encodings as single positions;
  equal runs give len_left x len_right pairs, the product Section 8 notes).

Blocks are listed by left entry, then right entry (the paper's Join Index
tensors are unsorted: any order of the same blocks is equally correct).
"""
from __future__ import annotations

import numpy as np

from . import oracle


def entries(col, n_rows, begin, end):
    """(values, starts, lengths) of a column's join entries inside [begin, end)."""
    enc = col["enc"]
    if enc == "rle":
        ends = np.asarray(col["run_ends"], dtype=np.int64)
        starts = np.concatenate([[0], ends[:-1]]).astype(np.int64)
        s = np.maximum(starts, begin)
        e = np.minimum(ends, end)
        keep = e > s
        return (np.asarray(col["values"], dtype=np.int64)[keep], s[keep], (e - s)[keep])
    if enc == "index":
        pos = np.asarray(col["positions"], dtype=np.int64)
        keep = (pos >= begin) & (pos < end)
        return (np.asarray(col["values"], dtype=np.int64)[keep], pos[keep], np.ones(int(keep.sum()), dtype=np.int64))
    vals = oracle.decode(col, n_rows)[begin:end].astype(np.int64)
    rows = np.arange(begin, end, dtype=np.int64)
    return vals, rows, np.ones(end - begin, dtype=np.int64)


def join_blocks(left, right):
    """Blocks (left_start, left_len, right_start, right_len) of two entry
    lists, by left entry, then right entry."""
    lv, ls, ll = left
    rv, rs, rl = right
    by_value = {}
    for j in range(len(rv)):
        by_value.setdefault(int(rv[j]), []).append(j)
    out = []
    for i in range(len(lv)):
        for j in by_value.get(int(lv[i]), ()):
            out.append((int(ls[i]), int(ll[i]), int(rs[j]), int(rl[j])))
    return out


def pairs(blocks):
    """The row pairs of a block list, block by block, left row outer."""
    out = []
    for a0, al, b0, bl in blocks:
        for a in range(a0, a0 + al):
            for b in range(b0, b0 + bl):
                out.append((a, b))
    return out


def apply(blocks, col, n_rows, side):
    """Apply Join Index: the values of `col` (an Index column holds 0 at the
    rows it does not list) at the `side` ("left" or "right") row of every
    pair, in pair order."""
    x = oracle.decode(col, n_rows).astype(np.int64)
    idx = [p[0] if side == "left" else p[1] for p in pairs(blocks)]
    return x[np.asarray(idx, dtype=np.int64)] if idx else np.zeros(0, dtype=np.int64)

"""CPU oracle of the composite-key (multi-attribute) sort and equi-join (test
infrastructure; shares no code with the GPU library).

A relation with key columns k_1 .. k_m is a set of points in an m-dimensional
key space; the sort orders them lexicographically (k_1 first), which is the
row-major linearisation of that space (Sec. III.B); the join matches rows
whose points coincide in every dimension (Sec. IV.A, a join condition over
several common attributes).

Definitions (plain, no blocking):
  sort:  the unique stable permutation p with (k_1[p(i)], ..., k_m[p(i)])
         non-decreasing lexicographically under signed comparison, ties kept
         in input order; keys_out[c][i] = k_c[p(i)], rids_out[i] = rid[p(i)].
  count: sum over distinct key tuples t of cnt_R(t) * cnt_S(t).
  pairs: every (rid_R[i], rid_S[j]) with equal tuples, ordered by tuple, then
         R position, then S position.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np


def _cols(cols):
    cols = [np.asarray(c) for c in cols]
    n = len(cols[0])
    for c in cols:
        if c.dtype not in (np.int32, np.int64) or len(c) != n:
            raise TypeError("key columns must be int32/int64 of equal length")
    return cols, n


def sort(cols, rids):
    """Stable lexicographic sort. numpy's lexsort is a stable sort keyed on the
    last array first, so the columns go in reverse."""
    cols, n = _cols(cols)
    if n == 0:
        return [c.copy() for c in cols], np.asarray(rids).copy()
    p = np.lexsort(tuple(c.astype(np.int64) for c in reversed(cols)))
    return [c[p] for c in cols], np.asarray(rids)[p]


def sort_loops(cols, rids):
    """The definition with Python tuples (small inputs): sort positions by
    (tuple, position)."""
    cols, n = _cols(cols)
    keyf = lambda i: tuple(int(c[i]) for c in cols) + (i,)
    p = sorted(range(n), key=keyf)
    return [c[p] for c in cols], np.asarray(rids)[p]


def join_count(r_cols, s_cols) -> int:
    r_cols, nr = _cols(r_cols)
    s_cols, ns = _cols(s_cols)
    cnt = defaultdict(int)
    for i in range(nr):
        cnt[tuple(int(c[i]) for c in r_cols)] += 1
    total = 0
    for j in range(ns):
        total += cnt.get(tuple(int(c[j]) for c in s_cols), 0)
    return total


def join_pairs(r_cols, r_rids, s_cols, s_rids):
    """Canonical pairs: tuple ascending, then R position, then S position."""
    r_cols, nr = _cols(r_cols)
    s_cols, ns = _cols(s_cols)
    rpos = defaultdict(list)
    for i in range(nr):
        rpos[tuple(int(c[i]) for c in r_cols)].append(i)
    spos = defaultdict(list)
    for j in range(ns):
        t = tuple(int(c[j]) for c in s_cols)
        if t in rpos:
            spos[t].append(j)
    out_r, out_s = [], []
    r_rids = np.asarray(r_rids)
    s_rids = np.asarray(s_rids)
    for t in sorted(spos):
        for i in rpos[t]:
            for j in spos[t]:
                out_r.append(r_rids[i])
                out_s.append(s_rids[j])
    return np.array(out_r, dtype=np.int32), np.array(out_s, dtype=np.int32), len(out_r)

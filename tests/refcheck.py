"""Independent reference computations used to pin the oracle.

None of this shares code with the oracle: brute-force nested loops, insertion
sort, numpy's stable argsort and a sort-merge counting formulation, plus the
invariant checks that hold at any size.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name: str) -> dict:
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            tag, *vals = line.split()
            out[tag] = [int(v) for v in vals]
    return out


def insertion_sort(keys, rids):
    """Stable insertion sort on Python ints (strict '>' keeps equal keys in order)."""
    out = []
    for k, r in zip(np.asarray(keys).tolist(), np.asarray(rids).tolist()):
        j = len(out)
        while j > 0 and out[j - 1][0] > k:
            j -= 1
        out.insert(j, (k, r))
    return [k for k, _ in out], [r for _, r in out]


def nested_loop_pairs(rk, rr, sk, sr):
    """All (key, i, j) with rk[i] == sk[j] by nested loops, sorted; returns rid lists."""
    rk, sk = np.asarray(rk).tolist(), np.asarray(sk).tolist()
    rr, sr = np.asarray(rr).tolist(), np.asarray(sr).tolist()
    trip = [(rk[i], i, j) for i in range(len(rk)) for j in range(len(sk)) if rk[i] == sk[j]]
    trip.sort()
    return [rr[i] for _, i, _ in trip], [sr[j] for _, _, j in trip]


def chunked_pairs(rk, rr, sk, sr, chunk: int = 1024):
    """Nested-loop join vectorised over row chunks; canonical order by lexsort."""
    rk, sk = np.asarray(rk), np.asarray(sk)
    ii, jj = [], []
    for i0 in range(0, rk.size, chunk):
        a, b = np.nonzero(rk[i0:i0 + chunk, None] == sk[None, :])
        ii.append(a + i0)
        jj.append(b)
    i = np.concatenate(ii) if ii else np.zeros(0, np.int64)
    j = np.concatenate(jj) if jj else np.zeros(0, np.int64)
    order = np.lexsort((j, i, rk[i]))  # primary key, then R position, then S position
    return np.asarray(rr)[i[order]], np.asarray(sr)[j[order]]


def chunked_count(rk, sk, chunk: int = 1024) -> int:
    rk, sk = np.asarray(rk), np.asarray(sk)
    total = 0
    for i0 in range(0, rk.size, chunk):
        total += int(np.count_nonzero(rk[i0:i0 + chunk, None] == sk[None, :]))
    return total


def sortmerge_count(rk, sk) -> int:
    """sum_k cnt_R(k) * cnt_S(k) from the two key histograms."""
    ur, cr = np.unique(np.asarray(rk), return_counts=True)
    us, cs = np.unique(np.asarray(sk), return_counts=True)
    _, ir, is_ = np.intersect1d(ur, us, assume_unique=True, return_indices=True)
    return int(np.sum(cr[ir].astype(object) * cs[is_].astype(object))) if ir.size else 0


def argsort_sort(keys, rids):
    order = np.argsort(np.asarray(keys), kind="stable")
    return np.asarray(keys)[order], np.asarray(rids)[order]


def check_sorted_permutation(keys_in, rids_in, keys_out, rids_out):
    """Invariants of a stable sort with rid = input position: keys ascend, every
    input row appears once with its own key, equal keys keep input order."""
    keys_in, keys_out = np.asarray(keys_in), np.asarray(keys_out)
    rids_out = np.asarray(rids_out)
    assert keys_out.size == keys_in.size
    assert np.all(keys_out[1:] >= keys_out[:-1]), "keys not ascending"
    pos = rids_out.astype(np.int64)
    assert np.array_equal(np.sort(pos), np.arange(keys_in.size)), "not a permutation"
    assert np.array_equal(keys_in[pos], keys_out), "row id does not carry its key"
    same = keys_out[1:] == keys_out[:-1]
    assert np.all(pos[1:][same] > pos[:-1][same]), "equal keys out of input order"

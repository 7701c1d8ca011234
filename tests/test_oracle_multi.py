"""Pins of the composite-key oracle (CPU only): the numpy path against the
tuple-loop definition, against brute-force nested loops, the one-column case
against the single-key oracle, and a two-column case against a packed single
key built by hand."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import multi


def _rel(rng, n, specs):
    return [rng.integers(lo, hi, n).astype(dt) for lo, hi, dt in specs]


SPECS = [
    [(-3, 3, np.int32), (0, 4, np.int64)],
    [(0, 2, np.int64), (-2, 2, np.int32), (0, 3, np.int32)],
    [(np.iinfo(np.int64).min, np.iinfo(np.int64).max, np.int64), (0, 2, np.int32)],
]


@pytest.mark.parametrize("spec", range(len(SPECS)))
def test_sort_matches_tuple_definition(spec):
    rng = np.random.default_rng(spec)
    cols = _rel(rng, 400, SPECS[spec])
    rids = rng.permutation(400).astype(np.int32)
    a_cols, a_r = multi.sort(cols, rids)
    b_cols, b_r = multi.sort_loops(cols, rids)
    assert np.array_equal(a_r, b_r)
    for x, y in zip(a_cols, b_cols):
        assert np.array_equal(x, y)
    # lexicographic, and stable: among equal tuples the input positions increase
    pos = np.argsort(rids)  # rid -> input position
    prev = None
    for i in range(400):
        t = tuple(int(c[i]) for c in a_cols)
        if prev is not None:
            assert prev[0] < t or (prev[0] == t and prev[1] < pos[a_r[i]])
        prev = (t, pos[a_r[i]])


def test_one_column_equals_single_key_oracle():
    rng = np.random.default_rng(4)
    k = rng.integers(-50, 50, 3000).astype(np.int64)
    r = rng.permutation(3000).astype(np.int32)
    (mk,), mr = multi.sort([k], r)
    ek, er = oracle.sort(k, r)
    assert np.array_equal(mk, ek) and np.array_equal(mr, er)
    s = rng.integers(-50, 50, 2000).astype(np.int64)
    sr = rng.permutation(2000).astype(np.int32)
    a = multi.join_pairs([k], r, [s], sr)
    b = oracle.join_pairs(k, r, s, sr)
    assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert multi.join_count([k], [s]) == oracle.join_count(k, s)


def test_join_brute_force():
    rng = np.random.default_rng(9)
    for spec in SPECS[:2]:
        rc = _rel(rng, 60, spec)
        sc = _rel(rng, 50, spec)
        rr = rng.permutation(60).astype(np.int32)
        sr = rng.permutation(50).astype(np.int32)
        got_r, got_s, cnt = multi.join_pairs(rc, rr, sc, sr)
        exp = []
        for i, j in itertools.product(range(60), range(50)):
            if all(int(a[i]) == int(b[j]) for a, b in zip(rc, sc)):
                exp.append((tuple(int(a[i]) for a in rc), i, j))
        exp.sort()
        assert cnt == len(exp) == multi.join_count(rc, sc)
        assert list(got_r) == [rr[i] for _, i, _ in exp] and list(got_s) == [sr[j] for _, _, j in exp]


def test_two_columns_against_packed_key():
    """(a, b) with a in [-8, 8), b in [0, 16): key = (a + 8) * 16 + b orders and
    matches exactly like the tuple."""
    rng = np.random.default_rng(12)
    ra, rb = rng.integers(-8, 8, 500).astype(np.int32), rng.integers(0, 16, 500).astype(np.int64)
    sa, sb = rng.integers(-8, 8, 700).astype(np.int32), rng.integers(0, 16, 700).astype(np.int64)
    rr, sr = np.arange(500, dtype=np.int32), np.arange(700, dtype=np.int32)
    pk_r = (ra.astype(np.int64) + 8) * 16 + rb
    pk_s = (sa.astype(np.int64) + 8) * 16 + sb
    (ga, gb), gr = multi.sort([ra, rb], rr)
    ek, er = oracle.sort(pk_r, rr)
    assert np.array_equal(gr, er) and np.array_equal((ga.astype(np.int64) + 8) * 16 + gb, ek)
    a = multi.join_pairs([ra, rb], rr, [sa, sb], sr)
    b = oracle.join_pairs(pk_r, rr, pk_s, sr)
    assert a[2] == b[2] and np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])

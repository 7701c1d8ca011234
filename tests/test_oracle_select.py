"""Pins of the path-selection oracle (oracle/pathsel.py) against published test
vectors, a brute-force bit-string reading of the register rule, the
HyperLogLog error bound on known cardinalities, and closed-form join sizes."""
import math

import numpy as np
import pytest

from oracle import pathsel as S

M = S.M
SIGMA = 1.04 / math.sqrt(M)  # the HyperLogLog standard error (Flajolet et al. 2007)


def _distinct(rng, d):
    keys = np.unique(rng.integers(-2**63, 2**63 - 1, size=int(d * 1.01) + 16, dtype=np.int64))[:d]
    rng.shuffle(keys)
    return keys


def test_hash_is_splitmix64_first_output():
    # A SplitMix64 generator seeded with s first outputs mix(s + gamma); seeded
    # with 0 its first three outputs are the published values below, i.e. the
    # hashes of the keys 0, gamma and 2 gamma (mod 2^64, read as int64).
    g = S.GAMMA
    expect = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    as_i64 = lambda x: x - 2**64 if x >= 2**63 else x
    keys = [as_i64((i * g) % 2**64) for i in range(3)]
    assert [S.hash64_scalar(k % 2**64) for k in keys] == expect
    assert [int(x) for x in S.hash64(np.array(keys, dtype=np.int64))] == expect


def test_hash_vector_matches_scalar_and_sign_extension():
    rng = np.random.default_rng(3)
    k64 = rng.integers(-2**63, 2**63 - 1, size=300, dtype=np.int64)
    assert [int(x) for x in S.hash64(k64)] == [S.hash64_scalar(int(k) % 2**64) for k in k64]
    k32 = rng.integers(-2**31, 2**31 - 1, size=300, dtype=np.int32)
    assert np.array_equal(S.hash64(k32), S.hash64(k32.astype(np.int64)))
    assert np.array_equal(S.registers(k32), S.registers(k32.astype(np.int64)))


def _brute_index_rank(h):
    bits = format(int(h), "064b")
    idx = int(bits[:S.M_BITS], 2)
    rest = bits[S.M_BITS:]
    rank = rest.index("1") + 1 if "1" in rest else len(rest) + 1
    return idx, rank


def test_index_rank_brute_force():
    rng = np.random.default_rng(5)
    hs = [0, 1, 2**49, 2**50 - 1, 2**50, 2**64 - 1, 2**63, 3 << 48] + \
        [int(x) for x in rng.integers(0, 2**64 - 1, size=2000, dtype=np.uint64)]
    # leading zeros of every length inside the 50 rank bits
    hs += [(int(rng.integers(0, 2**14)) << 50) | (1 << b) for b in range(50)]
    idx, rank = S.index_rank(np.array(hs, dtype=np.uint64))
    for h, i, r in zip(hs, idx, rank):
        assert (int(i), int(r)) == _brute_index_rank(h), hex(h)
    assert _brute_index_rank(0) == (0, 51) and _brute_index_rank(2**49) == (0, 1)


def test_registers_are_max_rank_per_index_brute_force():
    rng = np.random.default_rng(7)
    keys = rng.integers(-1000, 1000, size=3000, dtype=np.int64)
    reg = np.zeros(M, dtype=np.int64)
    for k in keys:
        i, r = _brute_index_rank(S.hash64_scalar(int(k) % 2**64))
        reg[i] = max(reg[i], r)
    assert np.array_equal(S.registers(keys), reg.astype(np.uint8))


@pytest.mark.parametrize("d", [1, 10, 1000, 20000, 50000, 200000, 2000000])
def test_estimate_within_error_bound(d):
    rng = np.random.default_rng(d)
    keys = _distinct(rng, d)
    # duplicates and order must not change the sketch
    dup = np.concatenate([keys, keys[: d // 3], keys[::7]])
    rng.shuffle(dup)
    reg = S.registers(keys)
    assert np.array_equal(S.registers(dup), reg)
    e = S.estimate(reg)
    if d <= 20000:  # linear-counting range: far tighter than the HLL bound
        assert abs(e - d) <= max(2.0, 0.01 * d), (d, e)
    else:
        assert abs(e - d) <= 3 * SIGMA * d, (d, e)


def test_estimate_special_cases():
    assert S.estimate(S.registers(np.zeros(0, dtype=np.int64))) == 0.0
    # one key: one register non-zero, linear counting m ln(m / (m - 1))
    assert S.estimate(S.registers(np.array([42], dtype=np.int64))) == M * math.log(M / (M - 1))
    # all registers at rank 1: Z = m / 2, raw estimate 2 alpha_m m (> 2.5 m is false: linear
    # counting applies only with empty registers, and there are none)
    reg = np.ones(M, dtype=np.uint8)
    alpha = 0.7213 / (1 + 1.079 / M)
    assert S.estimate(reg) == pytest.approx(2 * alpha * M, rel=1e-15)


def test_union_registers_are_those_of_the_concatenation():
    rng = np.random.default_rng(11)
    a = rng.integers(0, 10**6, size=50000, dtype=np.int64)
    b = rng.integers(5 * 10**5, 2 * 10**6, size=70000, dtype=np.int64)
    sel = S.select(a, b, min_rows=1)
    assert np.array_equal(sel["registers"][2], S.registers(np.concatenate([a, b])))
    true_union = np.unique(np.concatenate([a, b])).size
    assert abs(sel["distinct_union"] - true_union) <= 3 * SIGMA * true_union


def _exact_join(a, b):
    ka, ca = np.unique(a, return_counts=True)
    kb, cb = np.unique(b, return_counts=True)
    _, ia, ib = np.intersect1d(ka, kb, return_indices=True)
    return int((ca[ia].astype(np.int64) * cb[ib]).sum())


def test_join_estimate_closed_forms():
    rng = np.random.default_rng(13)
    d = 100000
    keys = _distinct(rng, d)
    # same distinct keys on both sides: output d
    sel = S.select(keys, rng.permutation(keys))
    assert abs(sel["est_output"] - d) <= 0.05 * d
    # foreign-key join: every S row matches one R row, output n_s
    s = keys[rng.integers(0, d, size=300000)]
    sel = S.select(keys, s)
    assert _exact_join(keys, s) == s.size
    assert abs(sel["est_output"] - s.size) <= 0.05 * s.size
    # every key 4 times in R and 3 times in S: output 12 d
    r4, s3 = np.repeat(keys, 4), np.repeat(keys, 3)
    sel = S.select(r4, s3)
    assert abs(sel["est_output"] - 12 * d) <= 0.05 * 12 * d
    assert abs(sel["distinct_common"] - d) <= 0.05 * d
    # disjoint key sets: no common keys, output near zero
    other = _distinct(np.random.default_rng(14), d)
    other = other[~np.isin(other, keys)]
    sel = S.select(keys, other)
    assert sel["distinct_common"] <= 0.05 * d and sel["est_output"] <= 0.05 * d
    # an empty side gives no output and no common keys
    sel = S.select(keys, keys[:0])
    assert sel["est_output"] == 0.0 and sel["distinct_common"] == 0.0 and sel["distinct_s"] == 0.0


def test_decision_rule():
    keys = np.arange(1000, dtype=np.int64)
    assert S.select(keys)["path"] == 0                           # small sort: linear
    sel = S.select(keys, min_rows=1000)
    assert (sel["path"], sel["reasons"]) == (1, 1)               # scale reached exactly
    sel = S.select(keys, min_rows=1001)
    assert (sel["path"], sel["reasons"]) == (0, 0)
    # a sort never takes the output reason; a join with a large expected output does
    many = np.repeat(np.arange(10, dtype=np.int64), 100)         # 10 keys x 100 rows
    sel = S.select(many, many, min_rows=10**9, min_output=50000)  # est ~ 10 * 100 * 100 = 1e5
    assert (sel["path"], sel["reasons"]) == (1, 2)
    sel = S.select(many, many, min_rows=2000, min_output=50000)
    assert (sel["path"], sel["reasons"]) == (1, 3)
    sel = S.select(many, many, min_rows=10**9, min_output=10**6)
    assert (sel["path"], sel["reasons"]) == (0, 0)
    # defaults
    assert S.select(np.arange(1 << 11, dtype=np.int64))["reasons"] == 1
    assert S.select(np.arange((1 << 11) - 1, dtype=np.int64))["reasons"] == 0

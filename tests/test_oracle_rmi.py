"""Pins of the learned-partitioner oracle (CPU only).

The bucket function must be non-decreasing in the key and stay in [0, F);
beyond that the pins tie each step of the fit to something other than the
oracle's own code: exact rational rounding for the integer-to-f32 conversion,
order statistics counted directly for the knots, numpy's least-squares
polynomial fit for the leaf models, and a closed form on an arithmetic
progression, where every leaf's points are collinear.
"""
from fractions import Fraction

import numpy as np
import pytest

import tjgen
from oracle import rmi


def _f32_exact_nearest(v: int) -> Fraction:
    """Nearest float32 to the integer v (ties to even), by exact arithmetic."""
    if v == 0:
        return Fraction(0)
    e = v.bit_length() - 24
    if e <= 0:
        return Fraction(v)
    q, r = divmod(v, 1 << e)
    half = 1 << (e - 1)
    if r > half or (r == half and q & 1):
        q += 1
    return Fraction(q << e)


def test_u64_to_f32_rounds_to_nearest_even():
    rng = np.random.default_rng(5)
    vals = [0, 1, (1 << 24) - 1, 1 << 24, (1 << 24) + 1, (1 << 25) + 1, (1 << 25) + 3, (1 << 62),
            (1 << 63) - 1, (1 << 64) - 1, (1 << 40) + (1 << 16), (1 << 40) + (1 << 16) + (1 << 17)]
    vals += [int(x) for x in rng.integers(0, 1 << 63, 2000, dtype=np.uint64)]
    vals += [int(x) >> int(s) for x, s in zip(rng.integers(0, 1 << 63, 2000, dtype=np.uint64),
                                              rng.integers(0, 60, 2000))]
    got = rmi.u64_to_f32(np.array(vals, dtype=np.uint64))
    for v, g in zip(vals, got):
        assert Fraction(float(g)) == _f32_exact_nearest(v), v


def test_i64_to_f32_sign_symmetric():
    v = np.array([-(1 << 62), -(1 << 40) - 12345, -3, 0, 3, (1 << 40) + 12345, 1 << 62], dtype=np.int64)
    f = rmi.i64_to_f32(v)
    assert np.array_equal(f, -rmi.i64_to_f32(-v))
    assert all(Fraction(float(x)) == (_f32_exact_nearest(int(a)) if a >= 0 else -_f32_exact_nearest(-int(a)))
               for x, a in zip(f, v))


def test_ordinals_preserve_signed_order():
    k = np.array([np.iinfo(np.int64).min, -5, -1, 0, 1, 7, np.iinfo(np.int64).max], dtype=np.int64)
    o = rmi.ordinals(k)
    assert (np.diff(o.astype(object)) > 0).all()
    k32 = np.array([np.iinfo(np.int32).min, -1, 0, 1, np.iinfo(np.int32).max], dtype=np.int32)
    o32 = rmi.ordinals(k32)
    assert (np.diff(o32.astype(object)) > 0).all() and int(o32.max()) < (1 << 32)


@pytest.mark.parametrize("n,permille", [(1, 10), (2048, 10), (2049, 10), (100_000, 10), (1_000_003, 10),
                                        (5000, 1000)])
def test_sample_positions(n, permille):
    p = rmi.sample_positions(n, permille)
    m = rmi.sample_count(n, permille)
    assert len(p) == m and p[0] == 0 and p[-1] < n and (np.diff(p) > 0).all()
    if n <= 2048:
        assert np.array_equal(p, np.arange(n))
    # evenly spread: position i lies in [i n / m, i n / m + 1)
    i = np.arange(m)
    assert np.all(p * m <= i * n) and np.all(i * n < (p + 1) * m)


def _keysets():
    rng = np.random.default_rng(11)
    out = {d: tjgen.learned(d, 1 << 18)["r_keys"] for d in tjgen.LEARNED_DISTS}
    out["uniform"] = rng.integers(-(1 << 62), 1 << 62, 1 << 18)
    out["dups"] = rng.integers(0, 50, 1 << 16) * (1 << 40)
    out["one_key"] = np.full(5000, -77, dtype=np.int64)
    out["extremes"] = np.concatenate([np.full(3000, np.iinfo(np.int64).min), np.full(3000, np.iinfo(np.int64).max),
                                      rng.integers(-10, 10, 3000)]).astype(np.int64)
    out["int32"] = rng.integers(-(1 << 31), 1 << 31, 1 << 17).astype(np.int32)
    out["tiny"] = np.array([3, 1, 2], dtype=np.int64)
    return out


@pytest.mark.parametrize("name", ["lognormal", "mixture", "seqgap", "uniform", "dups", "one_key", "extremes",
                                  "int32", "tiny"])
def test_bucket_monotone_and_in_range(name):
    k = _keysets()[name]
    m = rmi.train([k], buckets=512)
    o = np.sort(rmi.ordinals(k))
    # probe keys between and beyond the sample too
    ends = np.array([0, (1 << 64) - 1], dtype=np.uint64)
    probe = np.unique(np.concatenate([o, o[:-1] + (o[1:] - o[:-1]) // np.uint64(2), ends]))
    leaf = rmi.root_leaf(m, probe)
    b = rmi.bucket(m, probe)
    assert (np.diff(leaf) >= 0).all() and leaf.min() >= 0 and leaf.max() < rmi.LEAVES
    assert (np.diff(b) >= 0).all() and b.min() >= 0 and b.max() < 512
    # leaf intervals chain without overlap
    assert (m.leaf_lo <= m.leaf_hi).all() and (m.leaf_hi[:-1] <= m.leaf_lo[1:]).all()
    assert (m.leaf_b >= 0).all() and np.isfinite(m.leaf_a).all() and np.isfinite(m.leaf_b).all()


def test_knots_are_order_statistics():
    k = tjgen.learned("lognormal", 1 << 18)["r_keys"]
    m = rmi.train([k])
    s = rmi.ordinals(k)[rmi.sample_positions(len(k), 10)]
    M = len(s)
    assert m.sample_rows == M
    for i in range(rmi.SEGMENTS + 1):
        r = (i * (M - 1)) // rmi.SEGMENTS
        below = int((s < m.knot[i]).sum())
        upto = int((s <= m.knot[i]).sum())
        assert below <= r < upto
        if i < rmi.SEGMENTS:
            d = int(m.knot[i + 1]) - int(m.knot[i])
            if d:
                assert abs(float(m.knot_inv[i]) * d - 1.0) < 2.0 ** -22
            else:
                assert m.knot_inv[i] == 0


def test_leaf_fits_match_least_squares():
    k = tjgen.learned("mixture", 1 << 19)["r_keys"]
    m = rmi.train([k])
    s = np.sort(rmi.ordinals(k)[rmi.sample_positions(len(k), 10)])
    M = len(s)
    leaf = rmi.root_leaf(m, s)
    y = 512.0 * np.arange(M) / M
    checked = 0
    for l in np.unique(leaf):
        idx = np.nonzero(leaf == l)[0]
        if len(idx) < 3:
            continue
        base = s[idx[0]]
        d = (s[idx] - base).astype(np.float64)
        if d.max() == 0:
            continue
        assert m.leaf_base[l] == base
        slope, icpt = np.polyfit(d, y[idx], 1)
        slope = max(slope, 0.0)
        if slope == 0.0:
            icpt = y[idx].mean()
        assert float(m.leaf_b[l]) == pytest.approx(slope, rel=1e-5, abs=1e-30)
        assert float(m.leaf_a[l]) == pytest.approx(icpt, rel=1e-5, abs=1e-3)
        assert m.leaf_lo[l] == (512 * idx[0]) // M and m.leaf_hi[l] == (512 * idx[-1]) // M
        checked += 1
    assert checked > 100


def test_arithmetic_progression_closed_form():
    """Keys c + g i, all sampled (n <= 2048): every leaf's points are collinear, so
    each fit is exact and bucket(x_i) = floor(F i / n) up to one f32 rounding step."""
    n, c, g = 2048, -(1 << 50), 977
    i = np.arange(n)
    k = (c + g * i).astype(np.int64)
    perm = np.random.default_rng(3).permutation(n)
    m = rmi.train([k[perm]], buckets=512)
    b = rmi.bucket(m, rmi.ordinals(k))
    want = (512 * i) // n
    assert np.all(np.abs(b - want) <= 1)
    assert np.mean(b == want) > 0.95


def test_uniform_keys_give_balanced_buckets():
    # 2^22 keys: a 41,943-point sample, about 41 points per leaf
    k = np.random.default_rng(8).integers(0, 1 << 60, 1 << 22)
    m = rmi.train([k], buckets=512)
    c = np.bincount(rmi.bucket(m, rmi.ordinals(k)), minlength=512)
    assert c.max() < 1.6 * c.mean() and c.min() > 0.5 * c.mean()


def test_join_model_uses_both_relations():
    w = tjgen.learned("seqgap", 1 << 16)
    mj = rmi.train([w["r_keys"], w["s_keys"]])
    assert mj.sample_rows == 2 * rmi.sample_count(1 << 16, 10)
    # equal keys map to equal buckets in both relations (one function)
    kr = rmi.ordinals(w["r_keys"])
    ks = rmi.ordinals(w["s_keys"])
    common = np.intersect1d(kr, ks)[:1000]
    assert np.array_equal(rmi.bucket(mj, common), rmi.bucket(mj, common.copy()))

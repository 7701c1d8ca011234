"""Pivot splits of crowded buckets (GROUP_PIVOT), against the oracle.

A child bucket holding more than twice its share of its parent's rows (and
more than one leaf) is sampled at three rows; when two of them hold the same
key, the next pass splits the bucket around that key (below / equal / above)
instead of by a radix digit. The outputs must equal the oracle's whatever
the split; the tests also check that the split happens where it should
(stats["pivots"]) and not where the samples disagree.
"""
import numpy as np
import pytest

import oracle
import tjgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


def check_sort(tj, k, r, expect_pivots=None):
    ek, er = oracle.sort(k, r)
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True)
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(ro.cpu().numpy(), er)
    if expect_pivots is not None:
        assert expect_pivots(st["pivots"]), st
    return st


def check_join(tj, rk, rr, sk, sr, expect_pivots=None):
    exp_r, exp_s, cnt = oracle.join_pairs(rk, rr, sk, sr)
    pr, ps, st = tj.join(dev(rk), dev(rr), dev(sk), dev(sr), capacity=cnt, stats=True)
    assert pr.numel() == cnt
    assert np.array_equal(pr.cpu().numpy(), exp_r) and np.array_equal(ps.cpu().numpy(), exp_s)
    c, st2 = tj.join_count(dev(rk), dev(sk), stats=True)
    assert c == cnt
    if expect_pivots is not None:
        assert expect_pivots(st["pivots"]) and expect_pivots(st2["pivots"]), (st, st2)
    return st


def _hot_sort_keys(rng, n, hot, span_bits=40, dtype=np.int64):
    """n uniform keys over [0, 2^span_bits) plus `hot` = [(key, copies)], shuffled."""
    base = rng.integers(0, 1 << span_bits, n, dtype=np.int64)
    parts = [base] + [np.full(c, k, np.int64) for k, c in hot]
    k = np.concatenate(parts)
    rng.shuffle(k)
    return k.astype(dtype)


@pytest.mark.parametrize("dtype", [np.int64, np.int32])
def test_sort_hot_keys_split_around_pivot(tj, dtype):
    rng = np.random.default_rng(11)
    bits = 40 if dtype == np.int64 else 31
    hot = [(int(rng.integers(0, 1 << bits)), c) for c in (60_000, 30_000, 20_000, 12_000)]
    k = _hot_sort_keys(rng, 400_000, hot, bits, dtype)
    check_sort(tj, k, tjgen.perm_i32(k.size, 3), lambda p: p >= 1)


def test_sort_pivot_at_bucket_edges(tj):
    """The frequent key is its bucket's smallest key (the 'below' child is
    empty), then its largest (the 'above' child is empty)."""
    rng = np.random.default_rng(12)
    for where in ("min", "max"):
        k0 = 1 << 36
        near = rng.integers(1, 1 << 20, 20_000) * (1 if where == "min" else -1) + k0
        far = rng.integers(-(1 << 50), 1 << 50, 300_000)
        k = np.concatenate([far, near, np.full(120_000, k0)]).astype(np.int64)
        rng.shuffle(k)
        check_sort(tj, k, tjgen.perm_i32(k.size, 4), lambda p: p >= 1)


def test_sort_crowded_without_majority_takes_radix(tj):
    """A bucket crowded by a dense run of distinct keys: the samples disagree,
    so no pivot is taken and the radix digits finish the sort."""
    rng = np.random.default_rng(13)
    far = rng.integers(0, 1 << 40, 300_000)
    dense = (1 << 33) + rng.permutation(200_000)  # 200,000 distinct keys in one narrow run
    k = np.concatenate([far, dense]).astype(np.int64)
    rng.shuffle(k)
    check_sort(tj, k, tjgen.perm_i32(k.size, 5), lambda p: p == 0)


def test_sort_wide_keys_with_hot_key(tj):
    """Keys over the full 64-bit range: pivot passes on 8-byte keys next to
    radix passes, extremes included."""
    rng = np.random.default_rng(14)
    base = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, 300_000, dtype=np.int64)
    hot = np.array([np.iinfo(np.int64).min, -7, 123456789012345, np.iinfo(np.int64).max])
    k = np.concatenate([base] + [np.full(25_000, h) for h in hot]).astype(np.int64)
    rng.shuffle(k)
    check_sort(tj, k, tjgen.perm_i32(k.size, 6))


def test_join_hot_keys_split_around_pivot(tj):
    """Hot keys on both sides, 40-bit keys (narrowed to 4 bytes by the first
    pass): the split runs on narrowed keys and its single-key children become
    cross products."""
    rng = np.random.default_rng(15)
    rk = rng.choice(1 << 40, 150_000, replace=False).astype(np.int64)
    hot = rk[:6]
    rk = np.concatenate([rk, np.repeat(hot, [3, 1, 2, 1, 5, 1])])
    sk = np.concatenate([rk[rng.integers(0, rk.size, 300_000)],
                         np.repeat(hot, [40_000, 25_000, 15_000, 11_000, 9_500, 9_000]),
                         rng.integers(0, 1 << 40, 50_000)]).astype(np.int64)
    rng.shuffle(rk)
    rng.shuffle(sk)
    rr = rng.permutation(rk.size).astype(np.int32)
    sr = rng.permutation(sk.size).astype(np.int32)
    check_join(tj, rk, rr, sk, sr, lambda p: p >= 1)


def test_join_zipf_paper_shaped_with_pivots(tj):
    w = tjgen.hbm_scale(0.99, n_r=1 << 18, n_s=1 << 20, hot=1 << 11)
    rr = tjgen.perm_i32(1 << 18, 9)
    check_join(tj, w["r_keys"], rr, w["s_keys"], w["s_rids"], lambda p: p >= 1)


@pytest.mark.parametrize("budget", [1 << 20, 4 << 20])
def test_pivot_under_budget(tj, budget):
    """Budget-bound plans split crowded buckets too, inside the workspace
    window (rows packed at other offsets than in the output columns) and on
    the join's 4-byte range keys."""
    rng = np.random.default_rng(16)
    hot = [(int(rng.integers(0, 1 << 40)), c) for c in (60_000, 30_000, 12_000)]
    k = _hot_sort_keys(rng, 300_000, hot)
    r = tjgen.perm_i32(k.size, 7)
    ek, er = oracle.sort(k, r)
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, workspace_bytes=budget)
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(ro.cpu().numpy(), er)
    assert st["windows"] >= 1 and st["pivots"] >= 1, st
    w = tjgen.hbm_scale(0.99, n_r=1 << 17, n_s=1 << 19, hot=1 << 10)
    rr = tjgen.perm_i32(1 << 17, 10)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], rr, w["s_keys"], w["s_rids"])
    pr, ps, st = tj.join(dev(w["r_keys"]), dev(rr), dev(w["s_keys"]), dev(w["s_rids"]), capacity=cnt,
                         workspace_bytes=budget, stats=True)
    assert st["key_ranges"] > 1 or st["windows"] >= 1, st
    assert np.array_equal(pr.cpu().numpy(), exp_r) and np.array_equal(ps.cpu().numpy(), exp_s)


def _smallest_unlimited_budget(probe):
    """Smallest workspace (in 64 KiB steps) that still runs the one-range,
    window-free plan: the full data buffers with the smallest planner tables
    (256 leaf slots, 1024 children per launch)."""
    lo, hi = 1 << 16, 1 << 33
    while hi - lo > (1 << 16):
        mid = (lo + hi) // 2 // (1 << 16) * (1 << 16)
        st = probe(mid)
        if st is not None and st["key_ranges"] == 1 and st["windows"] == 0:
            hi = mid
        else:
            lo = mid
    return hi


def test_small_tables_list_large_children(tj):
    """Unlimited plans on the smallest planner tables: the device batching of a
    level overflows its 256 leaf slots, or lists children too large for a leaf
    next to the leaves it batched, many launches per level; the host plans the
    rest. Sort and join equal the oracle."""
    rng = np.random.default_rng(17)
    hot = [(int(rng.integers(0, 1 << 40)), c) for c in (40_000, 20_000, 15_000, 9_000)]
    k = _hot_sort_keys(rng, 600_000, hot)
    r = tjgen.perm_i32(k.size, 8)
    dk, dr = dev(k), dev(r)

    def probe_sort(ws):
        try:
            return tj.sort(dk, dr, workspace_bytes=ws, stats=True)[2]
        except tj.TjError:
            return None

    ws = _smallest_unlimited_budget(probe_sort)
    ek, er = oracle.sort(k, r)
    ko, ro, st = tj.sort(dk, dr, workspace_bytes=ws, stats=True)
    assert st["key_ranges"] == 1 and st["windows"] == 0 and st["pivots"] >= 1, st
    assert np.array_equal(ko.cpu().numpy(), ek) and np.array_equal(ro.cpu().numpy(), er)

    rk = rng.choice(1 << 40, 200_000, replace=False).astype(np.int64)
    sk = np.concatenate([rk[rng.integers(0, rk.size, 400_000)], np.repeat(rk[:3], [30_000, 12_000, 9_000])])
    rng.shuffle(sk)
    rr = rng.permutation(rk.size).astype(np.int32)
    sr = rng.permutation(sk.size).astype(np.int32)
    drk, dsk, drr, dsr = dev(rk), dev(sk), dev(rr), dev(sr)
    exp_r, exp_s, cnt = oracle.join_pairs(rk, rr, sk, sr)

    def probe_join(ws):
        try:
            return tj.join(drk, drr, dsk, dsr, capacity=cnt, workspace_bytes=ws, stats=True)[2]
        except tj.TjError:
            return None

    ws = _smallest_unlimited_budget(probe_join)
    pr, ps, st = tj.join(drk, drr, dsk, dsr, capacity=cnt, workspace_bytes=ws, stats=True)
    assert st["key_ranges"] == 1 and st["windows"] == 0, st
    assert np.array_equal(pr.cpu().numpy(), exp_r) and np.array_equal(ps.cpu().numpy(), exp_s)

"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Every comparison is bit-exact: sorted keys and row ids, join counts, and the
join pairs in canonical order (key, R position, S position).
"""
import numpy as np
import pytest

import oracle
import tjgen
from tests import refcheck as rc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

I64 = np.iinfo(np.int64)
I32 = np.iinfo(np.int32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


def check_sort(tj, keys, rids, **kw):
    ko, ro = tj.sort(dev(keys), dev(rids), **kw)
    ek, er = oracle.sort(keys, rids)
    gk, gr = host(ko), host(ro)
    assert np.array_equal(gk, ek), "keys differ at %s" % np.nonzero(gk != ek)[0][:5]
    assert np.array_equal(gr, er), "rids differ at %s" % np.nonzero(gr != er)[0][:5]


def check_join(tj, rk, rr, sk, sr, **kw):
    exp_r, exp_s, cnt = oracle.join_pairs(rk, rr, sk, sr)
    assert tj.join_count(dev(rk), dev(sk), **kw) == cnt
    pr, ps = tj.join(dev(rk), dev(rr), dev(sk), dev(sr), capacity=cnt, **kw)
    gr, gs = host(pr), host(ps)
    assert gr.size == cnt
    assert np.array_equal(gr, exp_r), "R rids differ at %s" % np.nonzero(gr != exp_r)[0][:5]
    assert np.array_equal(gs, exp_s), "S rids differ at %s" % np.nonzero(gs != exp_s)[0][:5]
    return cnt


# --------------------------------------------------------------------------- primitives

def test_wave_scan_dpp(tj):
    rng = np.random.default_rng(0)
    x = rng.integers(0, 1 << 20, 64 * 300).astype(np.int32)
    got = host(tj.tj.debug_wave_scan(dev(x))).astype(np.int64)
    exp = np.cumsum(x.reshape(-1, 64).astype(np.int64), axis=1).reshape(-1)
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("force_reorder", [False, True])
@pytest.mark.parametrize("bits,shift,skew", [(8, 0, False), (8, 12, False), (9, 55, False), (3, 40, False),
                                             (1, 5, False), (9, 55, True), (4, 60, True)])
def test_partition_pass(tj, bits, shift, skew, force_reorder):
    """One pass against a stable counting sort. force_reorder makes every tile
    take the scatter's re-ranking path as well; skew makes most rows share a
    few digits (long runs inside a tile)."""
    rng = np.random.default_rng(bits * 100 + shift)
    n = 100_003
    k = rng.integers(I64.min, I64.max, n, dtype=np.int64)
    if skew:
        k = rng.choice(k[:5], n)
    r = rng.integers(I32.min, I32.max, n, dtype=np.int32)
    ko, ro, counts = tj.tj.debug_partition_pass(dev(k), dev(r), 0, shift, bits, force_reorder=force_reorder)
    ordv = k.view(np.uint64) ^ np.uint64(1 << 63)
    digit = ((ordv >> np.uint64(shift)) & np.uint64((1 << bits) - 1)).astype(np.int64)
    order = np.argsort(digit, kind="stable")   # stable counting-sort partition
    assert np.array_equal(host(ko), k[order]) and np.array_equal(host(ro), r[order])
    assert np.array_equal(host(counts).astype(np.int64), np.bincount(digit, minlength=1 << bits))


# --------------------------------------------------------------------------- sort

def test_sort_small_uniform_int32(tj):
    w = tjgen.small_uniform()
    check_sort(tj, w["r_keys"], w["r_rids"])
    check_sort(tj, w["s_keys"], w["s_rids"])


@pytest.mark.parametrize("theta", [0.0, 0.99])
def test_sort_paper_shaped(tj, theta):
    w = tjgen.paper_shaped(theta, rid_perm=True)
    check_sort(tj, w["r_keys"], w["r_rids"])
    check_sort(tj, w["s_keys"], w["s_rids"])


def test_sort_uniform_64bit_keys(tj):
    w = tjgen.sort_uniform64(n=600_000)
    check_sort(tj, w["keys"], w["rids"])


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 4095, 4096, 4097, 8191, 8192, 8193, 9215, 9216, 9217, 16383, 16385, 18433, 20_000])
def test_sort_sizes(tj, n):
    rng = np.random.default_rng(n)
    k = rng.integers(-1000, 1000, n).astype(np.int64)
    r = rng.permutation(n).astype(np.int32)
    check_sort(tj, k, r)
    check_sort(tj, k.astype(np.int32), r)


@pytest.mark.parametrize("n", [4095, 4096, 4097, 8191, 8192, 8193, 12289, 40_000])
def test_sort_wide_key_leaf_sizes(tj, n):
    """Keys over the full 64-bit range (leaves span more than 32 bits), at
    sizes around one and two leaf blocks; also duplicated keys."""
    rng = np.random.default_rng(n + 7)
    k = rng.integers(I64.min, I64.max, n, dtype=np.int64)
    k[rng.integers(0, n, n // 16)] = k[rng.integers(0, n, n // 16)]
    check_sort(tj, k, rng.permutation(n).astype(np.int32))


def test_sort_wide_key_uneven_buckets(tj):
    """A multi-pass sort of 64-bit keys whose buckets differ widely in size:
    one dense region of the range gets buckets of thousands of rows next to
    buckets of a few hundred."""
    rng = np.random.default_rng(99)
    sparse = rng.integers(I64.min, I64.max, 300_000, dtype=np.int64)
    dense = rng.integers(-(1 << 50), 1 << 50, 400_000, dtype=np.int64)
    k = np.concatenate([sparse, dense])
    rng.shuffle(k)
    check_sort(tj, k, rng.permutation(k.size).astype(np.int32))


def test_sort_edge_distributions(tj):
    rng = np.random.default_rng(42)
    n = 50_000
    cases = {
        "all_equal": np.full(n, 7, np.int64),
        "two_keys": rng.choice(np.array([-5, 9]), n).astype(np.int64),
        "presorted": np.arange(n, dtype=np.int64) * 3,
        "reverse": (n - np.arange(n, dtype=np.int64)) * 1000003,
        "extremes": rng.choice(np.array([I64.min, I64.min + 1, -1, 0, 1, I64.max - 1, I64.max]), n),
        "hot_and_wide": np.where(rng.random(n) < 0.6, 123456789,
                                 rng.integers(I64.min, I64.max, n, dtype=np.int64)),
    }
    for name, k in cases.items():
        r = rng.permutation(n).astype(np.int32)
        check_sort(tj, k, r)
    check_sort(tj, np.array([I32.min, I32.max, -1, 0, I32.min], np.int32), np.arange(5, dtype=np.int32))


@pytest.mark.parametrize("distinct", [3, 40, 150, 700, 5000])
def test_sort_leaf_duplicates(tj, distinct):
    """One leaf-sized bucket with few distinct keys: with 40 distinct keys and
    fewer the one-pass bin sort sees bins above its limit and falls back to the
    digit passes; with more it ranks many equal keys inside each bin."""
    rng = np.random.default_rng(distinct)
    for n in (6000, 8192):
        vals = rng.integers(-(1 << 40), 1 << 40, distinct)
        k = rng.choice(vals, n).astype(np.int64)
        r = rng.permutation(n).astype(np.int32)
        check_sort(tj, k, r)
        check_sort(tj, (k >> 20).astype(np.int32), r)


def test_sort_empty(tj):
    ko, ro = tj.sort(dev(np.zeros(0, np.int64)), dev(np.zeros(0, np.int32)))
    assert ko.numel() == 0 and ro.numel() == 0


# --------------------------------------------------------------------------- join

def test_join_small_uniform_int32(tj):
    w = tjgen.small_uniform()
    cnt = check_join(tj, w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    assert cnt == rc.sortmerge_count(w["r_keys"], w["s_keys"])


@pytest.mark.parametrize("theta", [0.0, 0.99])
def test_join_paper_shaped(tj, theta):
    w = tjgen.paper_shaped(theta, rid_perm=True)
    assert check_join(tj, w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"]) == 800_000


def test_join_multiplicity_skew(tj):
    # hot keys with R multiplicity 4 and Zipf(0.99) S: several single-key buckets
    w = tjgen.hbm_scale(0.99, n_r=1 << 18, n_s=1 << 20, hot=1 << 12)
    assert check_join(tj, w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"]) == w.expected_count


@pytest.mark.parametrize("nr,ns", [(1, 1), (1, 5000), (5000, 1), (63, 65), (4097, 4095), (8193, 9000)])
def test_join_sizes(tj, nr, ns):
    rng = np.random.default_rng(nr * 7 + ns)
    for dom in (4, 300, 1 << 40):
        rk = rng.integers(0, dom, nr).astype(np.int64)
        sk = rng.integers(0, dom, ns).astype(np.int64)
        rr = rng.permutation(nr).astype(np.int32)
        sr = rng.permutation(ns).astype(np.int32)
        check_join(tj, rk, rr, sk, sr)


def test_join_edge_distributions(tj):
    rng = np.random.default_rng(5)
    # one hot key larger than a leaf block on both sides (cross-product path)
    rk = np.concatenate([np.full(9000, 77), rng.integers(0, 1000, 3000)]).astype(np.int64)
    sk = np.concatenate([np.full(12000, 77), rng.integers(0, 1000, 5000)]).astype(np.int64)
    rng.shuffle(rk)
    rng.shuffle(sk)
    rr = rng.permutation(rk.size).astype(np.int32)
    sr = rng.permutation(sk.size).astype(np.int32)
    check_join(tj, rk, rr, sk, sr)
    # negative and extreme keys, full 64-bit range
    ext = np.array([I64.min, I64.min + 1, -1, 0, 1, I64.max - 1, I64.max])
    rk = np.concatenate([rng.choice(ext, 3000), rng.integers(I64.min, I64.max, 3000, dtype=np.int64)])
    sk = np.concatenate([rng.choice(ext, 4000), rk[:1000]])
    check_join(tj, rk, np.arange(rk.size, dtype=np.int32), sk, np.arange(sk.size, dtype=np.int32))
    # no match at all
    rk = np.arange(0, 20000, 2, dtype=np.int64)
    sk = np.arange(1, 20000, 2, dtype=np.int64)
    assert check_join(tj, rk, np.arange(rk.size, dtype=np.int32), sk, np.arange(sk.size, dtype=np.int32)) == 0
    # int32 extremes
    rk = rng.choice(np.array([I32.min, -1, 0, I32.max], np.int32), 5000)
    sk = rng.choice(np.array([I32.min, 3, I32.max], np.int32), 700)
    check_join(tj, rk, np.arange(5000, dtype=np.int32), sk, np.arange(700, dtype=np.int32))


def test_join_capacity_contract(tj):
    w = tjgen.paper_shaped(0.5, n=50_000)
    rk, rr, sk, sr = dev(w["r_keys"]), dev(w["r_rids"]), dev(w["s_keys"]), dev(w["s_rids"])
    cnt = tj.join_count(rk, sk)
    assert cnt == 40_000
    with pytest.raises(tj.TjError) as e:
        tj.join(rk, rr, sk, sr, capacity=cnt - 1)
    assert e.value.status == -3
    pr, ps = tj.join(rk, rr, sk, sr, capacity=cnt)
    er, es, _ = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    assert np.array_equal(host(pr), er) and np.array_equal(host(ps), es)


@pytest.mark.parametrize("budget", [None, 4 << 20])
def test_join_mixed_key_widths(tj, budget):
    """Half the keys spread over the whole int64 range (their first-level
    buckets are leaves with 8-byte keys), half packed into a 2^36-wide range
    (one first-level bucket that is split again with keys narrowed to 4 bytes):
    one call runs leaves of both key widths, in key order."""
    rng = np.random.default_rng(36)
    n = 150_000
    sparse = rng.integers(I64.min, I64.max, n, dtype=np.int64)
    dense = (rng.integers(0, 1 << 36, n) + (5 << 50)).astype(np.int64)
    rk = np.concatenate([sparse, dense])
    rng.shuffle(rk)
    # S: 70% of its rows match R (some several times), the rest are fresh keys
    sk = np.concatenate([rng.choice(rk, 2 * n * 7 // 10),
                         rng.integers(I64.min, I64.max, 2 * n * 3 // 10, dtype=np.int64)])
    rng.shuffle(sk)
    rr = rng.permutation(rk.size).astype(np.int32)
    sr = rng.permutation(sk.size).astype(np.int32)
    kw = {} if budget is None else {"workspace_bytes": budget}
    check_join(tj, rk, rr, sk, sr, **kw)


def test_join_empty_sides(tj):
    k = dev(np.arange(10, dtype=np.int64))
    z = dev(np.zeros(0, np.int64))
    assert tj.join_count(k, z) == 0 and tj.join_count(z, k) == 0


# --------------------------------------------------------------------------- budgets

@pytest.mark.parametrize("theta", [0.0, 0.99])
@pytest.mark.parametrize("budget", [1 << 20, 64 << 20, None])
def test_budget_sweep_paper_shaped(tj, theta, budget):
    """Results are identical at 1 MiB, 64 MiB and an unlimited workspace."""
    w = tjgen.paper_shaped(theta, rid_perm=True)
    check_sort(tj, w["s_keys"], w["s_rids"], workspace_bytes=budget)
    cnt = check_join(tj, w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"], workspace_bytes=budget)
    assert cnt == 800_000


def test_budget_single_key_ranges(tj):
    # a hot key too large for a 1 MiB workspace on both sides
    rng = np.random.default_rng(8)
    rk = np.concatenate([np.full(60_000, 5), rng.integers(0, 1 << 30, 40_000)]).astype(np.int64)
    sk = np.concatenate([np.full(70_000, 5), np.full(3, 9), rng.integers(0, 1 << 30, 40_000)]).astype(np.int64)
    rng.shuffle(rk)
    rng.shuffle(sk)
    rr = rng.permutation(rk.size).astype(np.int32)
    sr = rng.permutation(sk.size).astype(np.int32)
    check_sort(tj, rk, rr, workspace_bytes=1 << 20)
    exp_r, exp_s, cnt = oracle.join_pairs(rk, rr, sk, sr)
    assert tj.join_count(dev(rk), dev(sk), workspace_bytes=1 << 20) == cnt
    # the pair output of the hot key alone is 4.2e9: check the count only, and
    # the pairs of a version where the hot key has few R rows
    rk2 = rk.copy()
    hot = np.nonzero(rk2 == 5)[0]
    rk2[hot[3:]] = 11
    exp_r, exp_s, cnt = oracle.join_pairs(rk2, rr, sk, sr)
    pr, ps = tj.join(dev(rk2), dev(rr), dev(sk), dev(sr), capacity=cnt, workspace_bytes=1 << 20)
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)


@pytest.mark.parametrize("name", ["uniform64", "lognormal", "zipf0.99"])
def test_budget_windowed_sort(tj, name):
    """Under a binding budget (8 MiB for 2^22 rows) the sort partitions into
    its output columns and finishes the buckets through the workspace window,
    a run of adjacent buckets at a time: several runs, with further passes
    inside the window; buckets larger than the window (the lognormal bulk, the
    hottest Zipf keys) are sorted the same way from the input filtered to
    their key range. Uniform keys are read from the input once. Results equal
    the oracle's."""
    n = 1 << 22
    if name == "uniform64":
        k = tjgen.uniform_i64(n, 77)
    elif name == "lognormal":
        k = tjgen.lognormal_i64(n, 78)
    else:
        k = tjgen.paper_shaped(0.99, n=n)["s_keys"]
    r = tjgen.perm_i32(n, 79)
    print("windowed sort %s n=%d" % (name, n), flush=True)
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, workspace_bytes=8 << 20)
    assert st["windows"] > 1, st
    if name == "uniform64":
        assert st["key_ranges"] == 1 and st["passes"] >= 2, st
    ek, er = oracle.sort(k, r)
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)


@pytest.mark.parametrize("n,bits,budget", [(1 << 21, 32, 2 << 20), (300_001, 12, 1 << 20), (70_000, 64, 1 << 20)])
def test_budget_sort_shapes(tj, n, bits, budget):
    """Budget-bound sorts beyond the int64 cases: int32 keys over the full
    range and over 2^12 values (every bucket a few keys, many single-key
    buckets already final in the output), and full-range int64 keys a little
    above the rows the 1 MiB window holds; against the oracle."""
    if bits == 64:
        k = tjgen.uniform_i64(n, 91)
    else:
        k = tjgen.uniform_i32(n, 92, bits)
    r = tjgen.perm_i32(n, 93)
    print("budget sort n=%d bits=%d budget=%d" % (n, bits, budget), flush=True)
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, workspace_bytes=budget)
    ek, er = oracle.sort(k, r)
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)
    assert st["key_ranges"] >= 1


@pytest.mark.parametrize("variant", ["window", "refilter"])
def test_budget_join_window(tj, variant):
    """Budget-bound join with 4-byte range keys: a key range whose bucket of
    three neighbouring keys (more rows than a leaf holds) needs another pass
    takes it through the workspace window, where its keys become single-key
    units that are output in key order among the range's other units
    ("window"); when that bucket has more rows than the window, it is read
    again from the input, filtered to its key range, into its own rows
    ("refilter"). Counts and pairs equal the oracle's."""
    rng = np.random.default_rng(21)
    n = 100_000
    base = rng.choice(1 << 40, n + 20_000, replace=False).astype(np.int64)
    k0 = (1 << 35) + 123456
    base = base[(base < k0 - 8) | (base > k0 + 8)]
    rk0, fresh = base[:n], base[n:]
    if variant == "window":
        hot_r = [1000, 1000, 2500]
        hot_s = [2500, 1000, 1000]
    else:
        hot_r = [6000, 5000, 4000]
        hot_s = [3000, 2000, 1000]
    rk = np.concatenate([rk0] + [np.full(c, k0 + i, np.int64) for i, c in enumerate(hot_r)])
    sk = np.concatenate([rk0[rng.integers(0, n, 80_000)], fresh[:20_000]] +
                        [np.full(c, k0 + i, np.int64) for i, c in enumerate(hot_s)])
    rng.shuffle(rk)
    rng.shuffle(sk)
    rr = rng.permutation(rk.size).astype(np.int32)
    sr = rng.permutation(sk.size).astype(np.int32)
    print("budget join window %s" % variant, flush=True)
    check_join(tj, rk, rr, sk, sr, workspace_bytes=1 << 20)
    pr, _, st = tj.join(dev(rk), dev(rr), dev(sk), dev(sr), workspace_bytes=1 << 20, stats=True)
    if variant == "window":
        assert st["windows"] >= 1, st
    else:
        assert st["key_ranges"] >= 2 and st["single_key"] >= 1, st


# --------------------------------------------------------------------------- profiling hook

def test_timing_hook_counts_launches(tj):
    w = tjgen.paper_shaped(0.0, n=100_000)
    rk, sk = dev(w["r_keys"]), dev(w["s_keys"])
    tj.timing(True)
    assert tj.join_count(rk, sk) == 80_000
    tj.timing(False)
    fams = tj.timing_read()
    assert fams["probe"]["launches"] == 1
    assert fams["leaf_join_count"]["launches"] >= 1 and fams["leaf_join_count"]["ms"] > 0
    assert fams["leaf_join_count"]["bytes"] >= 8 * 200_000
    tj.timing(True)  # re-enabling clears the counters
    assert all(v["launches"] == 0 for v in tj.timing_read().values())
    tj.timing(False)


def test_skewed_buckets_dominated_by_one_key(tj):
    # buckets where almost every row holds one key exercise the histogram's
    # wave-uniform path and the single-key detection at every depth
    rng = np.random.default_rng(17)
    n = 300_000
    k = np.where(rng.random(n) < 0.97, 1 << 35, rng.integers(0, 1 << 40, n)).astype(np.int64)
    r = rng.permutation(n).astype(np.int32)
    check_sort(tj, k, r)
    sk = np.where(rng.random(n) < 0.9, 1 << 35, rng.integers(0, 1 << 40, n)).astype(np.int64)
    rk = np.concatenate([np.full(3, 1 << 35), rng.integers(0, 1 << 40, 5000)]).astype(np.int64)
    check_join(tj, rk, np.arange(rk.size, dtype=np.int32), sk, r)


def test_sort_wide_keys_with_ties(tj):
    # 64-bit keys spread wide (wide leaves) with duplicated keys and keys that
    # share their high bits: the top-32-bit sort plus tie fix-up, and the
    # fall-back to the full sort when ties are many
    rng = np.random.default_rng(23)
    n = 400_000
    base = rng.integers(I64.min // 2, I64.max // 2, n // 4, dtype=np.int64)
    k = np.concatenate([base, base, base + rng.integers(0, 16, base.size), base ^ 1])
    rng.shuffle(k)
    check_sort(tj, k, rng.permutation(n).astype(np.int32))
    few = rng.choice(rng.integers(I64.min, I64.max, 7, dtype=np.int64), n)  # long tie runs
    check_sort(tj, few, np.arange(n, dtype=np.int32))


# --------------------------------------------------------------------------- fallback paths

def test_forced_reranking_paths(tj):
    """With TJ_DEBUG_FORCE_REORDER every partition tile and every join block
    also runs the ballot-ranked path that replaces an atomic-ranked order found
    out of input order: the results must be the same."""
    tj.tj.debug_set_flags(tj.tj.TJ_DEBUG_FORCE_REORDER)
    try:
        w = tjgen.paper_shaped(0.99, n=200_000, rid_perm=True)
        check_join(tj, w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
        check_sort(tj, w["s_keys"], w["s_rids"])
        rng = np.random.default_rng(11)
        k = rng.integers(-50, 50, 30_000).astype(np.int64)
        check_join(tj, k[:12_000], np.arange(12_000, dtype=np.int32), k[12_000:],
                   np.arange(18_000, dtype=np.int32))
        check_sort(tj, k, rng.permutation(k.size).astype(np.int32))
    finally:
        tj.tj.debug_set_flags(0)


@pytest.mark.parametrize("where", ["high", "low", "both"])
def test_sampled_range_miss(tj, where):
    """Large calls take their first digit range from every 4096th key. An
    outlier at an unsampled position falls outside it: the first histogram
    flags it and the call probes the exact range; results stay exact."""
    n = (1 << 22) + 3
    rng = np.random.default_rng(17)
    keys = rng.integers(0, 1 << 30, n).astype(np.int64)
    if where in ("high", "both"):
        keys[4097] = 1 << 50
    if where in ("low", "both"):
        keys[8191] = -(1 << 45)
    rids = tjgen.perm_i32(n, 9)
    check_sort(tj, keys, rids)
    s_keys = rng.integers(0, 1 << 30, n // 2).astype(np.int64)
    s_keys[1] = keys[4097]
    s_keys[2] = keys[8191]
    s_rids = tjgen.iota_i32(n // 2)
    cnt = oracle.join_count(keys, s_keys)
    assert tj.join_count(dev(keys), dev(s_keys)) == cnt
    pr, ps = tj.join(dev(keys), dev(rids), dev(s_keys), dev(s_rids), capacity=cnt)
    er, es, _ = oracle.join_pairs(keys, rids, s_keys, s_rids)
    assert np.array_equal(host(pr), er) and np.array_equal(host(ps), es)

"""GPU parity of the learned CDF partitioner.

Three layers, each against the CPU oracle:
  * the bucket function: the device evaluates an oracle-trained model on the
    keys and must give the oracle's bucket ids bit for bit (same f32
    operations, no fused multiply-add);
  * training: the device-trained model against the oracle-trained one on the
    same sample: integer fields and the knot inverses exactly, the fp64-fitted
    leaf lines to a few f32 ulps (their sums run in another order);
  * the sort and the join with the learned first pass: outputs identical to
    the oracle's sort order and canonical join pairs, as for the radix path.
"""
import numpy as np
import pytest

import oracle
import tjgen
from oracle import rmi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LEARN = dict(partitioner="learned", learned_min_rows=1)  # force the learned pass at test sizes


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


def _keys(name, n=1 << 18):
    rng = np.random.default_rng(31)
    if name in tjgen.LEARNED_DISTS:
        return tjgen.learned(name, n)["r_keys"]
    if name == "negative":
        return rng.integers(-(1 << 62), 1 << 40, n)
    if name == "extremes":
        return np.concatenate([np.full(n // 4, I64.min), np.full(n // 4, I64.max),
                               rng.integers(-5, 5, n // 2)]).astype(np.int64)
    if name == "dups":
        return (rng.integers(0, 300, n) * 7919).astype(np.int64)
    if name == "int32":
        return rng.integers(I32.min, I32.max, n, endpoint=True).astype(np.int32)
    raise ValueError(name)


I64 = np.iinfo(np.int64)
I32 = np.iinfo(np.int32)
KEYSETS = ["lognormal", "mixture", "seqgap", "negative", "extremes", "dups", "int32"]


@pytest.mark.parametrize("name", KEYSETS)
def test_bucket_function_bit_exact(tj, name):
    k = _keys(name)
    m = rmi.train([k], buckets=512)
    o = rmi.ordinals(k)
    # keys between sample points and beyond the extremes too
    probe_o = np.concatenate([o, o // np.uint64(2) + np.uint64(12345), np.array([0, (1 << 64) - 1], np.uint64)])
    if k.dtype == np.int32:
        probe_o = probe_o[probe_o < np.uint64(1 << 32)]
        probe = (probe_o.astype(np.uint32) ^ np.uint32(1 << 31)).view(np.int32)
    else:
        probe = (probe_o ^ np.uint64(1 << 63)).view(np.int64)
    got = host(tj.rmi_buckets(dev(probe), tj.RmiModel.from_fields(m)))
    exp = rmi.bucket(m, probe_o)
    bad = np.nonzero(got != exp)[0]
    assert bad.size == 0, "first mismatches at %s: got %s want %s" % (bad[:5], got[bad[:5]], exp[bad[:5]])


@pytest.mark.parametrize("name,join", [("lognormal", False), ("mixture", True), ("seqgap", True),
                                       ("dups", False), ("int32", False), ("extremes", False)])
def test_training_matches_oracle(tj, name, join):
    if join and name in tjgen.LEARNED_DISTS:
        w = tjgen.learned(name, 1 << 18)
        ka, kb = w["r_keys"], w["s_keys"]
    else:
        ka, kb = _keys(name), None
    exp = rmi.train([ka] if kb is None else [ka, kb], buckets=512)
    got = tj.rmi_train(dev(ka), None if kb is None else dev(kb)).to_numpy()
    assert got["buckets"] == 512 and got["sample_rows"] == exp.sample_rows
    for f in ("knot", "knot_inv", "leaf_base", "leaf_lo", "leaf_hi"):
        g, e = got[f], getattr(exp, f)
        assert np.array_equal(g, e), "%s differs at %s" % (f, np.nonzero(g != e)[0][:5])
    for f in ("leaf_a", "leaf_b"):
        g, e = got[f].astype(np.float64), getattr(exp, f).astype(np.float64)
        scale = np.maximum(np.abs(e), np.finfo(np.float32).tiny)
        assert np.all(np.abs(g - e) <= 4 * np.spacing(e.astype(np.float32)).astype(np.float64) + 1e-6 * scale), f
    # the device model is itself a valid monotone bucket function
    gm = tj.RmiModel.from_fields(got)
    srt = np.sort(ka)
    b = host(tj.rmi_buckets(dev(srt), gm))
    assert (np.diff(b) >= 0).all() and b.max() < 512


@pytest.mark.parametrize("name", KEYSETS)
def test_learned_sort_matches_oracle(tj, name):
    k = _keys(name, 300_001)
    r = tjgen.perm_i32(len(k), 77)
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, **LEARN)
    assert st["learned"] == 1 and st["sample_rows"] == rmi.sample_count(len(k), 10)
    ek, er = oracle.sort(k, r)
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)


@pytest.mark.parametrize("name", list(tjgen.LEARNED_DISTS))
@pytest.mark.parametrize("n", [20_000, 400_003])
def test_learned_join_matches_oracle(tj, name, n):
    w = tjgen.learned(name, n)
    rr = tjgen.perm_i32(n, 5)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], rr, w["s_keys"], w["s_rids"])
    c, st = tj.join_count(dev(w["r_keys"]), dev(w["s_keys"]), stats=True, **LEARN)
    assert c == cnt and st["learned"] == 1
    pr, ps, st = tj.join(dev(w["r_keys"]), dev(rr), dev(w["s_keys"]), dev(w["s_rids"]), capacity=cnt,
                         stats=True, **LEARN)
    assert st["learned"] == 1
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)


def test_learned_join_skewed_and_int32(tj):
    # Zipf(0.99) foreign keys: hot keys make single-key buckets in the learned pass
    w = tjgen.paper_shaped(0.99, n=300_000, rid_perm=True)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    pr, ps = tj.join(dev(w["r_keys"]), dev(w["r_rids"]), dev(w["s_keys"]), dev(w["s_rids"]), capacity=cnt,
                     **LEARN)
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)
    w = tjgen.small_uniform(n=200_000)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    pr, ps = tj.join(dev(w["r_keys"]), dev(w["r_rids"]), dev(w["s_keys"]), dev(w["s_rids"]), capacity=cnt,
                     **LEARN)
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)


def test_learned_falls_back_to_radix(tj):
    k = _keys("lognormal", 100_000)
    r = tjgen.iota_i32(len(k))
    ek, er = oracle.sort(k, r)
    # below the row threshold
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, partitioner="learned", learned_min_rows=1 << 20)
    assert st["learned"] == 0 and np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)
    # the minimum budget: key ranges, radix
    mn, full = tj.workspace_query(tj.TJ_OP_SORT, tj.TJ_KEY_I64, len(k))
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, workspace_bytes=mn, **LEARN)
    assert (st["key_ranges"] > 1 or st["windows"] > 0) and st["learned"] == 0
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)


@pytest.mark.parametrize("name", list(tjgen.LEARNED_DISTS))
def test_learned_equals_radix_large(tj, name):
    """2^24 rows per relation: learned and radix outputs identical; the learned
    pass leaves few buckets over twice the mean."""
    w = tjgen.learned(name, 1 << 24)
    rk, sk = dev(w["r_keys"]), dev(w["s_keys"])
    rid = dev(w["r_rids"])
    k1, r1, st1 = tj.sort(rk, rid, stats=True)
    k2, r2, st2 = tj.sort(rk, rid, stats=True, partitioner="learned")
    assert st2["learned"] == 1 and st1["learned"] == 0
    assert torch.equal(k1, k2) and torch.equal(r1, r2)
    assert st2["learned_overflow"] <= 8, st2
    c1 = tj.join_count(rk, sk)
    c2, st = tj.join_count(rk, sk, stats=True, partitioner="learned")
    assert c1 == c2 and st["learned"] == 1


@pytest.mark.parametrize("name,expect", [("lognormal", 1), ("mixture", 0), ("seqgap", 0)])
def test_auto_partitioner_decides_from_the_histogram(tj, name, expect):
    """Auto: lognormal keys put nearly all rows in one bucket of the radix
    digit (a heavy tail), so the call hands over to the learned pass; the
    interval mixture fills a few buckets, none with half the rows (its
    intervals split once the next level narrows the range), and gapped
    sequential keys spread evenly, so both stay radix. Results equal the radix
    path's either way."""
    w = tjgen.learned(name, 1 << 24)
    rk, sk, rid = dev(w["r_keys"]), dev(w["s_keys"]), dev(w["r_rids"])
    k1, r1 = tj.sort(rk, rid)
    k2, r2, st = tj.sort(rk, rid, stats=True, partitioner="auto")
    assert st["learned"] == expect, st
    assert torch.equal(k1, k2) and torch.equal(r1, r2)
    c, st = tj.join_count(rk, sk, stats=True, partitioner="auto")
    assert st["learned"] == expect and c == tj.join_count(rk, sk)


@pytest.mark.parametrize("name", list(tjgen.LEARNED_DISTS))
def test_auto_partitioner_matches_oracle(tj, name):
    w = tjgen.learned(name, 300_001)
    rr = tjgen.perm_i32(300_001, 3)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], rr, w["s_keys"], w["s_rids"])
    pr, ps = tj.join(dev(w["r_keys"]), dev(rr), dev(w["s_keys"]), dev(w["s_rids"]), capacity=cnt,
                     partitioner="auto", learned_min_rows=1)
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)
    ek, er = oracle.sort(w["r_keys"], rr)
    ko, ro = tj.sort(dev(w["r_keys"]), dev(rr), partitioner="auto", learned_min_rows=1)
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)

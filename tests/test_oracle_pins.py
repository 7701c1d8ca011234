"""Pins the CPU oracle to things other than itself (no GPU needed).

Sort (Sec. IV.B), join count and join pairs (Sec. IV.A) are checked against
hand-derived worked examples, brute-force nested loops, insertion sort, numpy's
stable argsort, a sort-merge count, closed-form join sizes that the generators
build in, and invariants. The mutation tests at the end rebuild the oracle with
a plausible mistake planted in a copy of its source and show that the pins
catch each one.
"""
import itertools
import os
import subprocess

import numpy as np
import pytest

import oracle
import tjgen
from tests import refcheck as rc

I64 = np.iinfo(np.int64)
I32 = np.iinfo(np.int32)


def _rand_keys(rng, n, domain, dtype):
    if domain == "full":
        info = np.iinfo(dtype)
        return rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)
    return rng.integers(-domain, domain, size=n).astype(dtype)


# --------------------------------------------------------------------------- golden

@pytest.mark.parametrize("name,dtype", [("join_tiny.txt", np.int64), ("join_tiny.txt", np.int32),
                                        ("extremes_i64.txt", np.int64)])
def test_golden_worked_examples(name, dtype):
    g = rc.load_golden(name)
    rk, sk = np.array(g["r_keys"], dtype), np.array(g["s_keys"], dtype)
    rr, sr = np.array(g["r_rids"], np.int32), np.array(g["s_rids"], np.int32)
    ko, ro = oracle.sort(rk, rr)
    assert ko.tolist() == g["sorted_r_keys"] and ro.tolist() == g["sorted_r_rids"]
    assert oracle.join_count(rk, sk) == g["count"][0]
    pr, ps, cnt = oracle.join_pairs(rk, rr, sk, sr)
    assert cnt == g["count"][0]
    assert pr.tolist() == g["pairs_r"] and ps.tolist() == g["pairs_s"]


# --------------------------------------------------------------------------- sort

def test_sort_exhaustive_tiny():
    # every key sequence of length <= 6 over {-1, 0, 1}
    for n in range(0, 7):
        for ks in itertools.product((-1, 0, 1), repeat=n):
            k = np.array(ks, dtype=np.int64)
            r = np.arange(n, dtype=np.int32)[::-1].copy()  # rids differ from positions
            ko, ro = oracle.sort(k, r)
            ek, er = rc.insertion_sort(k, r)
            assert ko.tolist() == ek and ro.tolist() == er


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("domain", [4, 64, 1 << 20, "full"])
def test_sort_matches_stable_argsort(dtype, domain):
    rng = np.random.default_rng(7)
    for n in (1, 2, 63, 64, 65, 1000, 20000):
        k = _rand_keys(rng, n, domain, dtype)
        r = rng.integers(I32.min, I32.max, size=n, dtype=np.int32)
        ko, ro = oracle.sort(k, r)
        ek, er = rc.argsort_sort(k, r)
        assert np.array_equal(ko, ek) and np.array_equal(ro, er)
        if n <= 1000:
            ik, ir = rc.insertion_sort(k, r)
            assert ko.tolist() == ik and ro.tolist() == ir


def test_sort_invariants_and_extremes():
    rng = np.random.default_rng(3)
    k = rng.choice(np.array([I64.min, I64.min + 1, -1, 0, 1, I64.max - 1, I64.max]), 5000)
    r = np.arange(k.size, dtype=np.int32)
    ko, ro = oracle.sort(k, r)
    rc.check_sorted_permutation(k, r, ko, ro)
    assert ko[0] == I64.min and ko[-1] == I64.max


def test_sort_small_uniform_workload():
    w = tjgen.small_uniform()
    ko, ro = oracle.sort(w["r_keys"], w["r_rids"])
    rc.check_sorted_permutation(w["r_keys"], w["r_rids"], ko, ro)
    ek, er = rc.argsort_sort(w["r_keys"], w["r_rids"])
    assert np.array_equal(ko, ek) and np.array_equal(ro, er)


# --------------------------------------------------------------------------- join

def test_join_exhaustive_tiny():
    # all R, S key sequences of length <= 3 over {-1, 0, 1}
    seqs = [s for n in range(4) for s in itertools.product((-1, 0, 1), repeat=n)]
    for rs in seqs:
        for ss in seqs:
            rk, sk = np.array(rs, np.int64), np.array(ss, np.int64)
            rr = np.arange(10, 10 + rk.size, dtype=np.int32)
            sr = np.arange(20, 20 + sk.size, dtype=np.int32)
            er, es = rc.nested_loop_pairs(rk, rr, sk, sr)
            assert oracle.join_count(rk, sk) == len(er)
            pr, ps, cnt = oracle.join_pairs(rk, rr, sk, sr)
            assert cnt == len(er) and pr.tolist() == er and ps.tolist() == es


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("domain", [3, 50, 1 << 12, "full"])
def test_join_matches_brute_force(dtype, domain):
    rng = np.random.default_rng(11)
    for nr, ns in ((0, 5), (5, 0), (1, 1), (300, 200), (2000, 3000)):
        rk, sk = _rand_keys(rng, nr, domain, dtype), _rand_keys(rng, ns, domain, dtype)
        rr = rng.integers(I32.min, I32.max, size=nr, dtype=np.int32)
        sr = rng.integers(I32.min, I32.max, size=ns, dtype=np.int32)
        er, es = rc.chunked_pairs(rk, rr, sk, sr)
        assert oracle.join_count(rk, sk) == er.size == rc.sortmerge_count(rk, sk)
        pr, ps, cnt = oracle.join_pairs(rk, rr, sk, sr)
        assert cnt == er.size and np.array_equal(pr, er) and np.array_equal(ps, es)
        if nr * ns <= 60000:
            nr_, ns_ = rc.nested_loop_pairs(rk, rr, sk, sr)
            assert pr.tolist() == nr_ and ps.tolist() == ns_


def test_join_capacity_prefix():
    rng = np.random.default_rng(5)
    rk, sk = rng.integers(0, 20, 500), rng.integers(0, 20, 500)
    rr, sr = np.arange(500, dtype=np.int32), np.arange(500, dtype=np.int32)
    full_r, full_s, cnt = oracle.join_pairs(rk, rr, sk, sr)
    pr, ps, cnt2 = oracle.join_pairs(rk, rr, sk, sr, capacity=cnt // 3)
    assert cnt2 == cnt and np.array_equal(pr, full_r[:cnt // 3]) and np.array_equal(ps, full_s[:cnt // 3])


def test_pairs_for_key_matches_join():
    rng = np.random.default_rng(9)
    rk, sk = rng.integers(0, 30, 400), rng.integers(0, 30, 600)
    rr = rng.permutation(400).astype(np.int32)
    sr = rng.permutation(600).astype(np.int32)
    pr, ps, _ = oracle.join_pairs(rk, rr, sk, sr)
    pos_r = {int(r): i for i, r in enumerate(rr)}
    pair_keys = np.array([rk[pos_r[int(r)]] for r in pr])
    for k in range(30):
        a, b = oracle.pairs_for_key(k, rk, rr, sk, sr)
        sel = pair_keys == k
        assert np.array_equal(a, pr[sel]) and np.array_equal(b, ps[sel])


def test_small_uniform_full_brute_force():
    # the whole 100,000 x 100,000 small workload by chunked nested loops
    w = tjgen.small_uniform()
    er, es = rc.chunked_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"], chunk=512)
    assert oracle.join_count(w["r_keys"], w["s_keys"]) == er.size
    pr, ps, cnt = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    assert np.array_equal(pr, er) and np.array_equal(ps, es)


@pytest.mark.parametrize("theta", [0.0, 0.99])
def test_paper_shaped_closed_form_count(theta):
    # R keys unique and 80% of S rows take an R key: |R join S| = 0.8 * |S| exactly
    w = tjgen.paper_shaped(theta)
    assert w.expected_count == 800_000
    assert oracle.join_count(w["r_keys"], w["s_keys"]) == 800_000
    assert rc.sortmerge_count(w["r_keys"], w["s_keys"]) == 800_000


def test_multiplicity_closed_form_count():
    # scaled-down skewed HBM construction: hot keys have R multiplicity 4
    w = tjgen.hbm_scale(theta=0.99, n_r=1 << 16, n_s=1 << 18, hot=1 << 10)
    assert oracle.join_count(w["r_keys"], w["s_keys"]) == w.expected_count
    assert rc.sortmerge_count(w["r_keys"], w["s_keys"]) == w.expected_count
    assert w.expected_count > 0.8 * (1 << 18)


# --------------------------------------------------------------------------- mutations

_MUTANTS = {
    # unsigned comparison instead of signed
    "unsigned_compare": ("return keys[a] < keys[b] || (keys[a] == keys[b] && a < b);",
                         "return (uint64_t)keys[a] < (uint64_t)keys[b] || (keys[a] == keys[b] && a < b);"),
    # ties broken against input order (unstable)
    "unstable_ties": ("(keys[a] == keys[b] && a < b)", "(keys[a] == keys[b] && a > b)"),
    # S-major emission within a key
    "s_major": ("for (uint64_t i : l.r)\n            for (uint64_t j : l.s) {",
                "for (uint64_t j : l.s)\n            for (uint64_t i : l.r) {"),
    # dropped multiplicity of R in the count
    "count_drops_mult": ("if (it != cnt_r.end()) total += it->second;",
                         "if (it != cnt_r.end()) total += 1;"),
    # descending key order of the pairs
    "keys_descending": ("std::sort(matched.begin(), matched.end());  // ascending key",
                        "std::sort(matched.rbegin(), matched.rend());"),
    # R and S rids swapped in the output
    "swapped_outputs": ("out_r[t] = r_rids[i];\n                    out_s[t] = s_rids[j];",
                        "out_r[t] = s_rids[j];\n                    out_s[t] = r_rids[i];"),
}


def _pins_pass(o: "oracle.Oracle") -> bool:
    try:
        for name, dtype in (("join_tiny.txt", np.int64), ("extremes_i64.txt", np.int64)):
            g = rc.load_golden(name)
            rk, sk = np.array(g["r_keys"], dtype), np.array(g["s_keys"], dtype)
            rr, sr = np.array(g["r_rids"], np.int32), np.array(g["s_rids"], np.int32)
            ko, ro = o.sort(rk, rr)
            assert ko.tolist() == g["sorted_r_keys"] and ro.tolist() == g["sorted_r_rids"]
            assert o.join_count(rk, sk) == g["count"][0]
            pr, ps, _ = o.join_pairs(rk, rr, sk, sr)
            assert pr.tolist() == g["pairs_r"] and ps.tolist() == g["pairs_s"]
        rng = np.random.default_rng(1)
        rk, sk = rng.integers(-5, 5, 300), rng.integers(-5, 5, 200)
        rr, sr = np.arange(300, dtype=np.int32), np.arange(200, dtype=np.int32)
        er, es = rc.chunked_pairs(rk, rr, sk, sr)
        pr, ps, cnt = o.join_pairs(rk, rr, sk, sr)
        assert o.join_count(rk, sk) == er.size
        assert np.array_equal(pr, er) and np.array_equal(ps, es)
        ko, ro = o.sort(rk, rr)
        ek, er2 = rc.argsort_sort(rk, rr)
        assert np.array_equal(ko, ek) and np.array_equal(ro, er2)
        return True
    except AssertionError:
        return False


def test_pins_accept_the_oracle():
    assert _pins_pass(oracle.Oracle(oracle.build()))


@pytest.mark.parametrize("mutant", sorted(_MUTANTS))
def test_pins_reject_planted_mistake(mutant, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "tj_oracle.cpp")).read()
    old, new = _MUTANTS[mutant]
    assert src.count(old) == 1, "mutation anchor not found exactly once"
    p = tmp_path / "mut.cpp"
    p.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-o", str(so), str(p)])
    assert not _pins_pass(oracle.Oracle(str(so)))

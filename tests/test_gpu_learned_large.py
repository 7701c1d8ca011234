"""GPU parity of the learned and auto partitioners at sizes where every
learned bucket is larger than one LDS block, so that each bucket takes radix
sub-passes seeded from the learned pass's per-bucket key ranges (the structure
the 2^28-row learned workload runs).

  * 2^22 / 2^23 rows: the whole output against the CPU oracle, bit for bit,
    for the three learned key distributions (learned forced) and for the
    auto partitioner.
  * 2^26 rows: properties that fix the result, computed with plain torch
    operations on the device: the stable sort (ordered, keys_out equal to
    keys_in at rids_out with rid = position, a permutation, ties in input
    order) and the canonical join (count equal to the sum over keys of
    cnt_R * cnt_S from torch's own sort and unique, every pair matching,
    strictly increasing in (key, R position, S position)), plus a few keys
    pair by pair against the oracle.
"""
import numpy as np
import pytest

import oracle
import tjgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LEARN = dict(partitioner="learned", learned_min_rows=1)


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.cpu().numpy()


def _lex_increasing(k, a, b):
    dk = k[1:] - k[:-1]
    if bool((dk < 0).any().item()):
        return False
    eqk = dk == 0
    del dk
    ok = (a[1:] > a[:-1]) | ((a[1:] == a[:-1]) & (b[1:] > b[:-1]))
    return bool((~eqk | ok).all().item())


def _torch_join_size(rk, sk):
    """sum over keys of cnt_R(k) * cnt_S(k), from torch's sort and unique."""
    ur, cr = torch.unique_consecutive(torch.sort(rk).values, return_counts=True)
    us, cs = torch.unique_consecutive(torch.sort(sk).values, return_counts=True)
    pos = torch.searchsorted(ur, us).clamp(max=ur.numel() - 1)
    hit = ur[pos] == us
    return int((cr[pos[hit]].to(torch.int64) * cs[hit].to(torch.int64)).sum().item())


@pytest.mark.parametrize("name", list(tjgen.LEARNED_DISTS))
def test_learned_sort_subpasses_match_oracle(tj, name):
    n = 1 << 23  # 16,384 rows per learned bucket on average: every bucket needs sub-passes
    w = tjgen.learned(name, n)
    k, r = w["r_keys"], tjgen.perm_i32(n, 41)
    print("learned sort %s n=%d" % (name, n), flush=True)
    ko, ro, st = tj.sort(dev(k), dev(r), stats=True, **LEARN)
    assert st["learned"] == 1 and st["passes"] >= 2, st
    ek, er = oracle.sort(k, r)
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)


@pytest.mark.parametrize("name", list(tjgen.LEARNED_DISTS))
def test_learned_join_subpasses_match_oracle(tj, name):
    n = 1 << 22  # per relation: 16,384 rows (R + S) per learned bucket on average
    w = tjgen.learned(name, n)
    rr = tjgen.perm_i32(n, 43)
    print("learned join %s n=%d" % (name, n), flush=True)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], rr, w["s_keys"], w["s_rids"])
    rk, sk = dev(w["r_keys"]), dev(w["s_keys"])
    c, st = tj.join_count(rk, sk, stats=True, **LEARN)
    assert c == cnt and st["learned"] == 1 and st["passes"] >= 2, st
    pr, ps, st = tj.join(rk, dev(rr), sk, dev(w["s_rids"]), capacity=cnt, stats=True, **LEARN)
    assert st["learned"] == 1
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)


@pytest.mark.parametrize("name", ["lognormal", "mixture"])
def test_auto_partitioner_large_matches_oracle(tj, name):
    n = 1 << 22
    w = tjgen.learned(name, n)
    rr = tjgen.perm_i32(n, 47)
    print("auto %s n=%d" % (name, n), flush=True)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], rr, w["s_keys"], w["s_rids"])
    pr, ps = tj.join(dev(w["r_keys"]), dev(rr), dev(w["s_keys"]), dev(w["s_rids"]), capacity=cnt,
                     partitioner="auto")
    assert np.array_equal(host(pr), exp_r) and np.array_equal(host(ps), exp_s)
    ek, er = oracle.sort(w["s_keys"], w["s_rids"])
    ko, ro = tj.sort(dev(w["s_keys"]), dev(w["s_rids"]), partitioner="auto")
    assert np.array_equal(host(ko), ek) and np.array_equal(host(ro), er)


@pytest.mark.parametrize("name", list(tjgen.LEARNED_DISTS))
def test_learned_properties_2e26(tj, name):
    n = 1 << 26
    w = tjgen.learned(name, n)
    print("learned properties %s n=%d" % (name, n), flush=True)
    d_rk, d_sk = dev(w["r_keys"]), dev(w["s_keys"])
    pos = torch.arange(n, dtype=torch.int32, device="cuda")
    # sort of R, rid = position
    ko, ro, st = tj.sort(d_rk, pos, stats=True, **LEARN)
    assert st["learned"] == 1 and st["passes"] >= 2, st
    assert bool((ko[1:] >= ko[:-1]).all().item()), "keys not ordered"
    assert torch.equal(d_rk[ro.long()], ko), "keys_out != keys_in[rids_out]"
    tie = ko[1:] == ko[:-1]
    assert bool((~tie | (ro[1:] > ro[:-1])).all().item()), "equal keys out of input order"
    seen = torch.zeros(n, dtype=torch.int8, device="cuda")
    seen[ro.long()] = 1
    assert int(seen.sum().item()) == n, "rids are not a permutation"
    del ko, ro, seen, tie
    # join, rid = position on both sides
    cnt = _torch_join_size(d_rk, d_sk)
    c, st = tj.join_count(d_rk, d_sk, stats=True, **LEARN)
    assert c == cnt and st["learned"] == 1, (c, cnt, st)
    pr, ps = tj.join(d_rk, pos, d_sk, pos, capacity=cnt, **LEARN)
    assert pr.numel() == cnt
    kr = d_rk[pr.long()]
    assert torch.equal(kr, d_sk[ps.long()]), "a pair joins different keys"
    assert _lex_increasing(kr, pr, ps), "pairs not in canonical order (or repeated)"
    rng = np.random.default_rng(5)
    r_rids = np.arange(n, dtype=np.int32)
    for i in rng.integers(0, cnt, 4):
        key = int(kr[int(i)].item())
        er, es = oracle.pairs_for_key(key, w["r_keys"], r_rids, w["s_keys"], r_rids)
        lo = int(torch.searchsorted(kr, torch.tensor([key], device="cuda")).item())
        hi = int(torch.searchsorted(kr, torch.tensor([key], device="cuda"), right=True).item())
        assert np.array_equal(host(pr[lo:hi]), er) and np.array_equal(host(ps[lo:hi]), es)

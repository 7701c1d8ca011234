"""Determinism across launch shapes and plans.

One input, run through every path that can produce a result, must give
bit-identical outputs:
  * the same call repeated, with other work on the device in between;
  * every partition tile and join block re-ranked by ballots
    (TJ_DEBUG_FORCE_REORDER) instead of LDS atomics;
  * the learned and the auto partitioner in place of the radix digit;
  * workspace budgets that bind (key ranges, workspace windows);
  * the sort on the library's static scratch;
  * the serving loop, with and without request fusion.
Every run is also equal to the oracle (one oracle call per input), so a
shared fault cannot make the runs agree with each other and pass.
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


def _sort_keys(n, seed):
    """Uniform 64-bit keys, a hot key, a dense narrow range and the extremes."""
    rng = np.random.default_rng(seed)
    k = rng.integers(-(1 << 62), 1 << 62, n, dtype=np.int64)
    pick = rng.random(n)
    k[pick < 0.2] = 987654321
    narrow = (pick >= 0.2) & (pick < 0.5)
    k[narrow] = rng.integers(0, 1 << 16, int(narrow.sum()))
    k[:3] = [np.iinfo(np.int64).min, np.iinfo(np.int64).max, -1]
    return k


def _reorder(tj, on):
    tj.tj.debug_set_flags(tj.tj.TJ_DEBUG_FORCE_REORDER if on else 0)


def test_sort_identical_across_plans(tj):
    n = 600_001
    k = _sort_keys(n, 5)
    r = tjgen.perm_i32(n, 6)
    ek, er = oracle.sort(k, r)
    dk, dr = dev(k), dev(r)
    runs = {}
    runs["default"] = tj.sort(dk, dr)
    noise = torch.randn(1 << 22, device="cuda")  # other device work between repeats
    runs["repeat"] = tj.sort(dk, dr)
    noise.mul_(2)
    _reorder(tj, True)
    try:
        runs["force_reorder"] = tj.sort(dk, dr)
    finally:
        _reorder(tj, False)
    runs["learned"] = tj.sort(dk, dr, partitioner="learned", learned_min_rows=1)
    runs["auto"] = tj.sort(dk, dr, partitioner="auto", learned_min_rows=1)
    mn, _ = tj.workspace_query(tj.TJ_OP_SORT, tj.TJ_KEY_I64, n)
    runs["min_workspace"] = tj.sort(dk, dr, workspace_bytes=mn)
    runs["1MiB"] = tj.sort(dk, dr, workspace_bytes=1 << 20)
    ko, ro = torch.empty_like(dk), torch.empty_like(dr)
    tj.sort_static(dk, dr, ko, ro)
    runs["static"] = (ko, ro)
    with tj.tj.Server(arena_bytes=256 << 20, slots=4) as srv:
        res = srv.wait(srv.sort(dk, dr))
        runs["server"] = (res["keys"], res["rids"])
        srv.configure(fuse_max_rows=1 << 20)
        t = [srv.sort(dk, dr) for _ in range(3)]
        for i, ti in enumerate(t):
            res = srv.wait(ti)
            runs["server_fused_%d" % i] = (res["keys"], res["rids"])
    torch.cuda.synchronize()
    base_k, base_r = runs["default"]
    assert np.array_equal(base_k.cpu().numpy(), ek) and np.array_equal(base_r.cpu().numpy(), er)
    for name, (kk, rr) in runs.items():
        assert torch.equal(kk, base_k) and torch.equal(rr, base_r), name


def test_join_identical_across_plans(tj):
    # hot R keys (x4) and Zipf(0.99) S keys: single-key buckets, crosses and
    # multi-level partitioning in one input
    w = tjgen.hbm_scale(0.99, n_r=1 << 17, n_s=1 << 19, hot=1 << 10)
    rr = tjgen.perm_i32(1 << 17, 8)
    exp_r, exp_s, cnt = oracle.join_pairs(w["r_keys"], rr, w["s_keys"], w["s_rids"])
    rk, sk, drr, dsr = dev(w["r_keys"]), dev(w["s_keys"]), dev(rr), dev(w["s_rids"])
    runs = {}
    runs["default"] = tj.join(rk, drr, sk, dsr, capacity=cnt)
    noise = torch.randn(1 << 22, device="cuda")
    runs["repeat"] = tj.join(rk, drr, sk, dsr, capacity=cnt)
    noise.mul_(2)
    _reorder(tj, True)
    try:
        runs["force_reorder"] = tj.join(rk, drr, sk, dsr, capacity=cnt)
    finally:
        _reorder(tj, False)
    runs["learned"] = tj.join(rk, drr, sk, dsr, capacity=cnt, partitioner="learned", learned_min_rows=1)
    runs["auto"] = tj.join(rk, drr, sk, dsr, capacity=cnt, partitioner="auto", learned_min_rows=1)
    runs["1MiB"] = tj.join(rk, drr, sk, dsr, capacity=cnt, workspace_bytes=1 << 20)
    runs["64MiB"] = tj.join(rk, drr, sk, dsr, capacity=cnt, workspace_bytes=64 << 20)
    with tj.tj.Server(arena_bytes=512 << 20, slots=4) as srv:
        res = srv.wait(srv.join(rk, drr, sk, dsr, capacity=cnt))
        runs["server"] = (res["out_r"], res["out_s"])
    torch.cuda.synchronize()
    base_r, base_s = runs["default"]
    assert base_r.numel() == cnt
    assert np.array_equal(base_r.cpu().numpy(), exp_r) and np.array_equal(base_s.cpu().numpy(), exp_s)
    for name, (a, b) in runs.items():
        assert torch.equal(a, base_r) and torch.equal(b, base_s), name
    counts = {tj.join_count(rk, sk), tj.join_count(rk, sk, workspace_bytes=1 << 20),
              tj.join_count(rk, sk, partitioner="learned", learned_min_rows=1)}
    assert counts == {cnt}

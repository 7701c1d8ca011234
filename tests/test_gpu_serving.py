"""GPU tests of the serving loop (tj_server_*).

Requests of uneven sizes, mixed operations and key distributions run
concurrently on several slots under a device-memory budget for their
workspaces; every result must be bit-identical to the same request run alone
through the plain calls, and to the CPU oracle. The budget is checked through
the server's peak arena use.
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


def _requests(count, seed, max_rows=200_000):
    """Mixed sort / join-count / join requests, log-uniform sizes, uniform or Zipf(0.8) keys."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(1000), np.log(max_rows))))
        op = ("sort", "join_count", "join")[i % 3]
        if rng.random() < 0.5:
            w = tjgen.paper_shaped(0.8, seed=seed * 1000 + i, n=n, rid_perm=True)
        else:
            w = tjgen.small_uniform(seed=seed * 1000 + i, n=n, bits=int(rng.integers(12, 30)), rid_perm=True)
        part = "learned" if rng.random() < 0.25 else "radix"
        out.append((op, w, part))
    return out


def _alone(tj, op, d, part):
    if op == "sort":
        return tj.sort(d["r_keys"], d["r_rids"], partitioner=part)
    if op == "join_count":
        return tj.join_count(d["r_keys"], d["s_keys"], partitioner=part)
    return tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], partitioner=part)


def _submit(srv, op, d, part, capacity=0):
    if op == "sort":
        return srv.sort(d["r_keys"], d["r_rids"], partitioner=part)
    if op == "join_count":
        return srv.join_count(d["r_keys"], d["s_keys"], partitioner=part)
    return srv.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=capacity, partitioner=part)


def _cap(op, w):
    return oracle.join_count(w["r_keys"], w["s_keys"]) if op == "join" else 0


def _check_oracle(op, w, res):
    if op == "sort":
        ek, er = oracle.sort(w["r_keys"], w["r_rids"])
        assert np.array_equal(res["keys"].cpu().numpy(), ek) and np.array_equal(res["rids"].cpu().numpy(), er)
    elif op == "join_count":
        assert res["count"] == oracle.join_count(w["r_keys"], w["s_keys"])
    else:
        er, es, cnt = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
        assert res["count"] == cnt
        assert np.array_equal(res["out_r"].cpu().numpy(), er) and np.array_equal(res["out_s"].cpu().numpy(), es)


@pytest.mark.parametrize("slots", [1, 4, 8])
def test_results_same_alone_and_in_mix(tj, slots):
    reqs = _requests(30, seed=slots)
    devs = [{k: dev(v) for k, v in w.items()} for _, w, _ in reqs]
    alone = [_alone(tj, op, d, part) for (op, _, part), d in zip(reqs, devs)]
    torch.cuda.synchronize()
    with tj.tj.Server(2 << 30, slots=slots) as srv:
        tickets = [_submit(srv, op, d, part, _cap(op, w)) for (op, w, part), d in zip(reqs, devs)]
        for (op, w, part), t, a in zip(reqs, tickets, alone):
            res = srv.wait(t)
            assert res["status"] == 0, res
            if op == "sort":
                assert torch.equal(res["keys"], a[0]) and torch.equal(res["rids"], a[1])
            elif op == "join_count":
                assert res["count"] == a
            else:
                assert torch.equal(res["out_r"], a[0]) and torch.equal(res["out_s"], a[1])
            _check_oracle(op, w, res)
        used, peak = srv.memory()
        assert used == 0 and 0 < peak <= 2 << 30


def test_admission_under_a_tight_budget(tj):
    """A 6 MiB arena cannot hold every request's full workspace at once:
    requests wait for memory, larger ones run with the minimum workspace (key
    ranges), the peak stays within the arena, and a request whose smallest
    workspace exceeds it fails alone with TJ_E_WORKSPACE."""
    arena = 6 << 20
    reqs = _requests(16, seed=99, max_rows=400_000)
    devs = [{k: dev(v) for k, v in w.items()} for _, w, _ in reqs]
    with tj.tj.Server(arena, slots=4) as srv:
        tickets = [_submit(srv, op, d, part, _cap(op, w)) for (op, w, part), d in zip(reqs, devs)]
        # a request nothing can hold: its minimum workspace alone is larger than the arena
        tiny = tj.tj.Server(256 << 10, slots=1)
        tb = tiny.sort(devs[0]["r_keys"], devs[0]["r_rids"])
        assert tiny.wait(tb)["status"] == tj.tj.TJ_E_WORKSPACE
        tiny.close()
        ranges = 0
        for (op, w, part), t in zip(reqs, tickets):
            res = srv.wait(t)
            assert res["status"] == 0, res
            ranges += res["key_ranges"] > 1 or res["windows"] > 0
            _check_oracle(op, w, res)
        used, peak = srv.memory()
        assert used == 0 and peak <= arena
    assert ranges > 0, "the tight budget never bound (no key ranges, no windowed sort)"


def test_capacity_and_wait_errors(tj):
    w = tjgen.paper_shaped(0.0, n=20_000, rid_perm=True)
    d = {k: dev(v) for k, v in w.items()}
    cnt = oracle.join_count(w["r_keys"], w["s_keys"])
    with tj.tj.Server(64 << 20, slots=2) as srv:
        t = srv.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=cnt - 1)
        res = srv.wait(t)
        assert res["status"] == tj.tj.TJ_E_CAPACITY and res["count"] == cnt
        with pytest.raises(tj.TjError):
            srv.wait(t)  # a ticket is forgotten once waited for


def test_many_small_requests_overlap(tj):
    """200 small sorts on 8 slots: all correct, and the busiest moment had more
    than one request on the GPU (their slot intervals overlap)."""
    w = tjgen.paper_shaped(0.8, n=30_000, rid_perm=True)
    d = {k: dev(v) for k, v in w.items()}
    ek, er = oracle.sort(w["s_keys"], w["s_rids"])
    with tj.tj.Server(512 << 20, slots=8) as srv:
        ts = [srv.sort(d["s_keys"], d["s_rids"]) for _ in range(200)]
        res = [srv.wait(t) for t in ts]
    for r in res:
        assert r["status"] == 0
        assert np.array_equal(r["keys"].cpu().numpy(), ek) and np.array_equal(r["rids"].cpu().numpy(), er)
    # requests queued behind others spent time waiting; the sum of slot times
    # exceeds the span of the whole batch only if slots ran at once
    span = max(r["total_ms"] for r in res)
    busy = sum(r["run_ms"] for r in res)
    assert busy > span, (busy, span)


def _small_requests(count, seed):
    """Small sorts and joins (0 .. 30,000 rows per side), int32 and int64 keys,
    uniform or Zipf(0.8), permuted row ids: all below the fusion threshold."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(0, 30_000)) if i % 7 else int(rng.integers(0, 3))
        op = "sort" if i % 2 else "join"
        if i % 3 == 0:
            w = tjgen.small_uniform(seed=seed * 1000 + i, n=n, bits=int(rng.integers(8, 24)), rid_perm=True)
        else:
            w = tjgen.paper_shaped(0.8 if i % 4 else 0.0, seed=seed * 1000 + i, n=n, rid_perm=True)
        out.append((op, w))
    return out


@pytest.mark.parametrize("slots", [1, 3])
def test_fused_small_requests_match_alone(tj, slots):
    """Small requests that queue up behind a large one are served by fused
    calls (one composite-key call per batch): every result equals the request
    run alone and the oracle, and batches of more than one request formed."""
    reqs = _small_requests(96, seed=5 + slots)
    devs = [{k: dev(v) for k, v in w.items()} for _, w in reqs]
    alone = [_alone(tj, op, d, "radix") for (op, _), d in zip(reqs, devs)]
    big = tjgen.sort_uniform64(1 << 24)["keys"]
    d_big = dev(big)
    d_big_r = torch.arange(big.size, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with tj.tj.Server(2 << 30, slots=slots) as srv:
        blockers = [srv.sort(d_big, d_big_r) for _ in range(slots)]  # keep every slot busy meanwhile
        tickets = [_submit(srv, op, d, "radix", _cap(op, w)) for (op, w), d in zip(reqs, devs)]
        for t in blockers:
            assert srv.wait(t)["status"] == 0
        fused = []
        for (op, w), t, a in zip(reqs, tickets, alone):
            res = srv.wait(t)
            assert res["status"] == 0, res
            fused.append(res["fused"])
            if op == "sort":
                assert torch.equal(res["keys"], a[0]) and torch.equal(res["rids"], a[1])
            else:
                assert torch.equal(res["out_r"], a[0]) and torch.equal(res["out_s"], a[1])
            _check_oracle(op, w, res)
        assert srv.memory()[0] == 0
    assert max(fused) > 1, fused


def test_fused_batch_with_a_short_capacity(tj):
    """One join of a fused batch has capacity for one pair less than it
    needs: it reports TJ_E_CAPACITY with its count and writes nothing at or
    beyond its capacity; the other requests of the batch are unaffected."""
    reqs = _small_requests(12, seed=11)
    reqs = [(op, w) for op, w in reqs if op == "join" and len(w["r_keys"]) > 100]
    devs = [{k: dev(v) for k, v in w.items()} for _, w in reqs]
    caps = [oracle.join_count(w["r_keys"], w["s_keys"]) for _, w in reqs]
    assert caps[0] > 0
    guard = 1 << 16
    outs = []
    with tj.tj.Server(1 << 30, slots=1) as srv:
        tickets = []
        for i, ((op, w), d) in enumerate(zip(reqs, devs)):
            cap = caps[i] - 1 if i == 0 else caps[i]
            o_r = torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda")
            o_s = torch.full((cap + guard,), -7, dtype=torch.int32, device="cuda")
            outs.append((o_r, o_s, cap))
            tickets.append(srv.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=cap,
                                    out_r=o_r, out_s=o_s))
        for i, ((op, w), t) in enumerate(zip(reqs, tickets)):
            res = srv.wait(t)
            o_r, o_s, cap = outs[i]
            assert bool((o_r[cap:] == -7).all().item()) and bool((o_s[cap:] == -7).all().item())
            if i == 0:
                assert res["status"] == tj.tj.TJ_E_CAPACITY and res["count"] == caps[0]
            else:
                assert res["status"] == 0
                _check_oracle(op, w, res)


def test_fusion_can_be_turned_off(tj):
    reqs = _small_requests(24, seed=13)
    devs = [{k: dev(v) for k, v in w.items()} for _, w in reqs]
    with tj.tj.Server(1 << 30, slots=2) as srv:
        srv.configure(0)
        tickets = [_submit(srv, op, d, "radix", _cap(op, w)) for (op, w), d in zip(reqs, devs)]
        for (op, w), t in zip(reqs, tickets):
            res = srv.wait(t)
            assert res["status"] == 0 and res["fused"] == 1
            _check_oracle(op, w, res)
        with pytest.raises(tj.TjError):
            srv.configure(1 << 16, 1000)  # more requests per call than allowed

"""Benchmark of the tensor-path sort and equi-join on one MI355X.

A step is one pass of the whole hot path over one batch of resident input:
  tj_sort of the standalone sort relation, then tj_join_materialize of R and S
  (range probe, radix histograms, scans, stable scatters, per-bucket LDS sorts
  and joins, pair materialisation).
Default workload (HBM scale): |R| = 2^27, |S| = 2^29 int64 keys with int32 row
ids (unique R keys over [0, 2^40), S foreign-key style, 80% matching,
uniform), plus a standalone sort of 2^29 (int64 key, int32 rid) rows with keys
uniform over the full 64-bit range. Inputs are generated on the host from fixed
seeds and are resident in HBM before timing starts.

value = (sort rows + |R| + |S|) / step time  [tuples/s], whole job.
roofline: the kernel family with the most time; algorithmic bytes per launch
over its HIP-event-measured average duration, against the 8 TB/s HBM peak.
cpu_baseline: the CPU oracle (single thread) on a 1/32 sample of the workload;
beside it the oracle built -O3 -march=native on this host and pinned to one
core: P50/P99 of C1 and of the paper-shaped workload, and the sort and join
times of the path-selection sweep (2^8 ... 2^22 rows per side), from which the
size where the tensor path overtakes it is read.
paper_shaped: P50/P99 latency of the |R| = |S| = 10^6 workload at workspace
budgets of 1 MiB, 64 MiB and unlimited, theta in {0, 0.99}.
learned_vs_radix: |R| = |S| = 2^28 int64 keys from a lognormal, an interval
mixture and a gapped sequence; sort, join count and join of the same inputs
with the radix, the learned and the auto first pass (median of 5), outputs
equal.
composite_keys: sort and join on two key columns, 2^26 rows per relation,
packed into one key (60 bits) or wide (128 bits: LSD groups / dense ranks).
path_selection: the execution-time selector (HyperLogLog sketch of the join
and sort keys) on the step's inputs, its indicators against the exact counts,
and the join latency of the tensor path from 2^10 to 2^22 rows per side with
the decision taken at each size.
stream_copy: a hand-written 16-byte streaming copy of 4 GiB, the bandwidth a
read-once write-once kernel reaches (the practical ceiling beside the peak).
c1_small: |R| = |S| = 10^5 int32 keys uniform in [0, 2^20): GPU P50/P99 of the
sort and the join over 100 calls.
hbm_zipf: the HBM-scale join with Zipf(0.99) matches (hot keys with
multiplicity 4, 1.37e9 pairs) and a sort of its 2^29 skewed S keys, timed
like the step, with its kernel families and roofline; plus the standalone sort
of 2^29 keys uniform over [0, 2^40).
serving: Poisson arrivals at 50, 200, 800 and 3200 requests/s of sorts and joins
(per-side rows log-uniform in [10^3, 10^7]) against the serving loop with a
32 GiB workspace budget, 8 slots against one at a time: P50/P99/P99.9 latency
and tuples/s, every result compared with the same request run alone.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "join input tuples/s + sort keys/s (%HBM peak); P50/P99 latency; learned vs radix"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


class no_gc:
    """Python's cyclic collector off while a timed loop runs: a collection
    inside a timed call (several ms with torch loaded) is not the library's
    time."""

    def __enter__(self):
        gc.collect()
        gc.disable()

    def __exit__(self, *exc):
        gc.enable()


def kernel_source_digest() -> str:
    """Short SHA-256 of the kernel sources; a traffic record taken on other
    sources no longer describes the kernels that run."""
    import hashlib
    h = hashlib.sha256()
    for f in ("tj_kernels.hip", "tj_internal.h"):
        with open(os.path.join(ROOT, "paper_2602_21237_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(family: str, workload: str):
    """HBM bytes per launch of a kernel family, from the committed summary of
    two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by a plain copy of
    known size. Returns (bytes or None, reason)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (family, workload))
    if not os.path.exists(path):
        return None, "no counter summary for this kernel"
    rec = None
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("traffic-record: "):
                rec = json.loads(ln[len("traffic-record: "):])
    if rec is None:
        return None, "summary has no traffic-record line"
    if rec.get("kernel_source_sha256_16") != kernel_source_digest():
        return None, "kernel sources changed since the counters were taken"
    return int(rec["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)


def pct(xs, q):
    """Nearest-rank percentile: sorted ascending, x[ceil(q*m) - 1]."""
    xs = sorted(xs)
    k = max(1, int(np.ceil(q * len(xs))))
    return xs[k - 1]


def make_workload(kind: str, theta: float):
    import tjgen
    if kind == "hbm":
        w = tjgen.hbm_scale(theta)
        sort_keys = tjgen.sort_uniform64(1 << 29)["keys"]
        desc = ("hbm_scale: join |R|=2^27 x |S|=2^29 int64 keys (unique R keys in [0,2^40), "
                "S 80%% FK matches, Zipf theta=%g) + standalone sort of 2^29 int64 keys uniform "
                "over 64 bits; int32 row ids" % theta)
    elif kind == "paper":
        w = tjgen.paper_shaped(theta)
        sort_keys = w["s_keys"]
        desc = "paper_shaped: |R|=|S|=10^6 int64 keys, theta=%g; sort of S" % theta
    elif kind == "small":
        w = tjgen.small_uniform()
        sort_keys = w["r_keys"]
        desc = "small_uniform: |R|=|S|=10^5 int32 keys uniform in [0,2^20); sort of R"
    else:
        raise SystemExit("unknown workload " + kind)
    return w, sort_keys, desc


def cpu_baseline(kind: str, theta: float):
    """The oracle, untuned, on a bounded sample of the same workload."""
    import oracle
    import tjgen
    if kind == "hbm":
        frac = 32
        w = tjgen.hbm_scale(theta, n_r=(1 << 27) // frac, n_s=(1 << 29) // frac,
                            hot=(1 << 20) // frac if theta > 0 else 0)
        sk = tjgen.sort_uniform64((1 << 29) // frac)["keys"]
        sample = ("1/32 of the workload: sort of 2^24 uniform 64-bit keys + join of "
                  "2^22 x 2^24 rows, same generators")
    else:
        w, sk, _ = make_workload(kind, theta)
        sample = "the whole workload"
    rids = np.arange(sk.size, dtype=np.int32)
    t0 = time.perf_counter()
    oracle.sort(sk, rids)
    t1 = time.perf_counter()
    oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    t2 = time.perf_counter()
    tuples = sk.size + w["r_keys"].size + w["s_keys"].size
    return {"value": tuples / (t2 - t0), "unit": "tuples/s", "cores": 1, "kind": "oracle",
            "sample": sample, "seconds": round(t2 - t0, 3), "sort_s": round(t1 - t0, 3),
            "join_s": round(t2 - t1, 3), "host_cpus": os.cpu_count()}


def paper_shaped_sweep(tj, torch, repeats: int):
    """P50/P99 of sort and join at N = 10^6 for three workspace budgets."""
    import tjgen
    out = {}
    for theta in (0.0, 0.99):
        w = tjgen.paper_shaped(theta)
        d = {k: torch.from_numpy(v).to("cuda") for k, v in w.items()}
        cap = 800_000
        out_r = torch.empty(cap, dtype=torch.int32, device="cuda")
        out_s = torch.empty(cap, dtype=torch.int32, device="cuda")
        ko = torch.empty_like(d["s_keys"])
        ro = torch.empty_like(d["s_rids"])
        for name, budget in (("1MiB", 1 << 20), ("64MiB", 64 << 20), ("unlimited", None)):
            res = {}
            for op in ("sort", "join"):
                if budget is None:
                    opc = tj.TJ_OP_SORT if op == "sort" else tj.TJ_OP_JOIN_MATERIALIZE
                    wsb = tj.workspace_query(opc, tj.TJ_KEY_I64, 10 ** 6, 10 ** 6)[1]
                else:
                    wsb = budget
                ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
                times = []
                st = None
                for i in range(repeats + 5):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    if op == "sort":
                        _, _, st = tj.sort(d["s_keys"], d["s_rids"], keys_out=ko, rids_out=ro,
                                           workspace=ws, stats=True)
                    else:
                        _, _, st = tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"],
                                           capacity=cap, out_r=out_r, out_s=out_s, workspace=ws,
                                           stats=True)
                    torch.cuda.synchronize()
                    if i >= 5:
                        times.append((time.perf_counter() - t0) * 1e3)
                res[op] = {"p50_ms": round(pct(times, 0.5), 3), "p99_ms": round(pct(times, 0.99), 3),
                           "key_ranges": st["key_ranges"],
                           "planned_MB": round((st["bytes_read"] + st["bytes_written"]) / 1e6, 1)}
                del ws
            out["theta%g_%s" % (theta, name)] = res
        del d, out_r, out_s, ko, ro
        torch.cuda.empty_cache()
    return out


def learned_vs_radix(tj, torch, n: int, repeats: int):
    """Radix against learned first-pass partitioning on the three non-uniform key
    distributions (|R| = |S| = n, int64 keys): sort of R, join count and join
    materialisation of R and S, same inputs, outputs checked equal."""
    import tjgen
    out = {}
    for dist in tjgen.LEARNED_DISTS:
        log("learned vs radix: generating %s, n = %d" % (dist, n))
        w = tjgen.learned(dist, n)
        rk = torch.from_numpy(w["r_keys"]).to("cuda")
        sk = torch.from_numpy(w["s_keys"]).to("cuda")
        rr = torch.from_numpy(w["r_rids"]).to("cuda")
        sr = torch.from_numpy(w["s_rids"]).to("cuda")
        del w
        ws_sort = torch.empty(tj.workspace_query(tj.TJ_OP_SORT, tj.TJ_KEY_I64, n)[1], dtype=torch.uint8,
                              device="cuda")
        ws_join = torch.empty(tj.workspace_query(tj.TJ_OP_JOIN_MATERIALIZE, tj.TJ_KEY_I64, n, n)[1],
                              dtype=torch.uint8, device="cuda")
        outs = {}
        res = {}
        count = tj.join_count(rk, sk, workspace=ws_join)
        mat = count < (1 << 30)
        if mat:
            out_r = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
            out_s = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
        for mode in ("radix", "learned", "auto"):
            ko, ro = torch.empty_like(rk), torch.empty_like(rr)
            ops = {"sort": lambda: tj.sort(rk, rr, keys_out=ko, rids_out=ro, workspace=ws_sort, stats=True,
                                           partitioner=mode)[2],
                   "join_count": lambda: tj.join_count(rk, sk, workspace=ws_join, stats=True,
                                                       partitioner=mode)[1]}
            if mat:
                ops["join"] = lambda: tj.join(rk, rr, sk, sr, capacity=count, out_r=out_r, out_s=out_s,
                                              workspace=ws_join, stats=True, partitioner=mode)[2]
            for op, f in ops.items():
                f()  # warm-up
                tj.timing(True)
                times = []
                for _ in range(repeats):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st = f()
                    torch.cuda.synchronize()
                    times.append((time.perf_counter() - t0) * 1e3)
                tj.timing(False)
                fams = tj.timing_read()
                r = res.setdefault(op, {})
                r[mode + "_ms"] = round(pct(times, 0.5), 3)
                r[mode + "_passes"] = st["passes"]
                r[mode + "_planned_MB"] = round((st["bytes_read"] + st["bytes_written"]) / 1e6, 1)
                r[mode + "_kernels_ms"] = {k: round(v["ms"] / repeats, 3) for k, v in fams.items() if v["launches"]}
                if mode == "auto":
                    r["auto_chose"] = "learned" if st["learned"] else "radix"
                    r["auto_speedup"] = round(r["radix_ms"] / r["auto_ms"], 3)
                if mode == "learned":
                    r["learned_ran"] = bool(st["learned"])
                    r["learned_overflow_buckets"] = st["learned_overflow"]
                    r["sample_rows"] = st["sample_rows"]
                    r["speedup"] = round(r["radix_ms"] / r["learned_ms"], 3)
            if mat:
                outs[mode] = (ko, ro, out_r[:count].clone(), out_s[:count].clone())
            else:
                outs[mode] = (ko, ro)
        same = all(torch.equal(a, b) for m in ("learned", "auto") for a, b in zip(outs["radix"], outs[m]))
        assert same, "learned and radix outputs differ (%s)" % dist
        res["join_count_value"] = count
        res["outputs_identical"] = same
        out[dist] = res
        log("learned vs radix %s: sort %.2f -> %.2f ms, join count %.2f -> %.2f ms" %
            (dist, res["sort"]["radix_ms"], res["sort"]["learned_ms"], res["join_count"]["radix_ms"],
             res["join_count"]["learned_ms"]))
        del rk, sk, rr, sr, ws_sort, ws_join, outs
        if mat:
            del out_r, out_s
        torch.cuda.empty_cache()
    return {"n_per_relation": n, "repeats": repeats, "dists": out}


def serving(tj, torch, rates, nreq: int, pool: int = 64, arena_gib: int = 32, slots: int = 8,
            saturate: bool = True):
    """Poisson stream of sort and join requests against the serving loop.

    Pool: `pool` requests resident on the GPU, per-side rows log-uniform in
    [10^3, 10^7], int64 keys (R keys unique over [0, 2^40), S foreign keys with
    Zipf(0) or Zipf(0.8) over R's keys, half each), op sort (of S) or join
    (materialised pairs), half each. Each rate runs `nreq` arrivals (seeded
    exponential gaps; pool entries drawn uniformly) in three modes: `slots`
    concurrent slots with fusion of small requests (the default), the same
    without fusion (rates of 800/s and more), and one request at a time (one
    slot, no fusion). Latency runs from the scheduled arrival to completion. With
    `saturate`, all `nreq` arrive at once as well: requests per second over the
    makespan is the highest rate each mode sustains on this mix. Every result is
    compared with the same request run alone."""
    import threading
    import tjgen
    rng = np.random.default_rng(2602)
    reqs = []
    log("serving: generating %d pooled requests" % pool)
    for i in range(pool):
        n_r = int(np.exp(rng.uniform(np.log(1e3), np.log(1e7))))
        n_s = int(np.exp(rng.uniform(np.log(1e3), np.log(1e7))))
        theta = 0.8 if i % 2 else 0.0
        w = tjgen._fk_pair(100 + i, n_r, n_s, theta)
        d = {k: torch.from_numpy(v).to("cuda") for k, v in w.items()}
        op = "sort" if (i // 2) % 2 else "join"
        e = {"op": op, "d": d, "tuples": n_s if op == "sort" else n_r + n_s}
        if op == "sort":
            e["ref"] = tj.sort(d["s_keys"], d["s_rids"])
            e["out"] = (torch.empty_like(d["s_keys"]), torch.empty_like(d["s_rids"]))
        else:
            e["count"] = w.expected_count
            e["ref"] = tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=e["count"])
            e["out"] = (torch.empty(max(e["count"], 1), dtype=torch.int32, device="cuda"),
                        torch.empty(max(e["count"], 1), dtype=torch.int32, device="cuda"))
        reqs.append(e)
        if (i + 1) % 32 == 0:
            log("serving: %d of %d pooled requests ready" % (i + 1, pool))
    torch.cuda.synchronize()
    rows = [e["tuples"] for e in reqs]
    out = {"pool": pool, "requests_per_rate": nreq, "arena_GiB": arena_gib, "slots": slots,
           "pool_mean_rows": round(float(np.mean(rows)), 1), "rates": {}}

    def run(sched, order, nslots, fuse):
        srv = tj.tj.Server(arena_gib << 30, slots=nslots)
        if not fuse:
            srv.configure(0)
        # warm-up: every slot's first call sets up its host-side staging
        warm = [srv.sort(reqs[i % pool]["d"]["s_keys"], reqs[i % pool]["d"]["s_rids"])
                for i in range(1, 4 * nslots, 4)]
        for t in warm:
            srv.wait(t)
        busy = set()
        lock = threading.Lock()
        done = []
        tickets = []  # (ticket, entry, scheduled time, submit delay)
        cv = threading.Condition()

        def waiter():
            k = 0
            while k < nreq:
                with cv:
                    while len(tickets) <= k:
                        cv.wait()
                    t, ei, ts, delay = tickets[k]
                r = srv.wait(t)
                e = reqs[ei]
                ok = r["status"] == 0
                if ok and e["op"] == "sort":
                    ok = torch.equal(r["keys"], e["ref"][0]) and torch.equal(r["rids"], e["ref"][1])
                elif ok:
                    ok = torch.equal(r["out_r"], e["ref"][0]) and torch.equal(r["out_s"], e["ref"][1])
                with lock:
                    busy.discard(ei)
                done.append((delay + r["total_ms"], r["queue_ms"], r["run_ms"], ok, e["tuples"],
                             ts * 1e3 + delay + r["total_ms"], r["fused"]))
                k += 1
                if k % 2000 == 0:
                    log("serving: %d of %d requests done" % (k, nreq))

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for i in range(nreq):
            ei = int(order[i])
            while True:  # an entry's output buffers serve one request at a time
                with lock:
                    free = [x for x in range(pool) if (ei + x) % pool not in busy]
                    if free:
                        ei = (ei + free[0]) % pool
                        busy.add(ei)
                        break
                time.sleep(0.0005)  # every entry in flight: the arrival waits (counted in its latency)
            now = time.perf_counter() - t0
            if sched[i] > now:
                time.sleep(sched[i] - now)
            delay = (time.perf_counter() - t0 - sched[i]) * 1e3
            e = reqs[ei]
            d = e["d"]
            if e["op"] == "sort":
                t = srv.sort(d["s_keys"], d["s_rids"], keys_out=e["out"][0], rids_out=e["out"][1])
            else:
                t = srv.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=e["count"],
                             out_r=e["out"][0], out_s=e["out"][1])
            with cv:
                tickets.append((t, ei, sched[i], delay))
                cv.notify()
        th.join()
        peak = srv.memory()[1]
        srv.close()
        lat = [x[0] for x in done]
        makespan_ms = max(x[5] for x in done)
        tuples = sum(x[4] for x in done)
        fused = [x[6] for x in done]
        assert all(x[3] for x in done), "a served result differs from the same request run alone"
        return {"p50_ms": round(pct(lat, 0.5), 3), "p99_ms": round(pct(lat, 0.99), 3),
                "p999_ms": round(pct(lat, 0.999), 3), "mean_ms": round(float(np.mean(lat)), 3),
                "tuples_per_s": round(tuples / (makespan_ms * 1e-3), 1),
                "requests_per_s": round(nreq / (makespan_ms * 1e-3), 1),
                "mean_queue_ms": round(float(np.mean([x[1] for x in done])), 3),
                "mean_run_ms": round(float(np.mean([x[2] for x in done])), 3),
                "fused_requests_frac": round(float(np.mean([f > 1 for f in fused])), 4),
                "max_fused_batch": int(max(fused)),
                "peak_arena_GB": round(peak / 1e9, 3), "results_identical": True}

    cases = [(r, "%g" % r) for r in rates] + ([(float("inf"), "saturated")] if saturate else [])
    for rate, name in cases:
        if np.isinf(rate):
            sched = np.zeros(nreq)
        else:
            gaps = np.random.default_rng(int(rate)).exponential(1.0 / rate, nreq)
            sched = np.cumsum(gaps) - gaps[0]
        order = np.random.default_rng(7 if np.isinf(rate) else int(rate) + 1).integers(0, pool, nreq)
        modes = [("served", slots, True)]
        if rate >= 800:
            modes.append(("served_no_fusion", slots, False))
        modes.append(("one_at_a_time", 1, False))
        res_rate = {}
        for mode, nslots, fuse in modes:
            res_rate[mode] = r = run(sched, order, nslots, fuse)
            log("serving %s %s: P50 %.2f P99 %.2f P99.9 %.2f ms, %.1f req/s, %.3g tuples/s, %.1f%% fused" %
                (name, mode, r["p50_ms"], r["p99_ms"], r["p999_ms"], r["requests_per_s"], r["tuples_per_s"],
                 100 * r["fused_requests_frac"]))
        out["rates"][name] = res_rate
    if saturate:
        out["max_sustainable_requests_per_s"] = {m: v["requests_per_s"]
                                                 for m, v in out["rates"]["saturated"].items()}
    del reqs
    torch.cuda.empty_cache()
    return out


def composite_keys(tj, torch, n: int, repeats: int = 3):
    """Composite-key sort (n rows) and join (n x n rows) through tj_*_multi:
    'packed' = an int32 column in [0, 2^20) and an int64 column in [0, 2^40)
    (60 bits: one 8-byte sort key); 'wide' = two int64 columns over the full
    range (128 bits: two stable sorts; the join through dense ranks). S copies
    the tuples of uniformly chosen R rows for 80% of its rows."""
    rng = np.random.default_rng(31)
    specs = {"packed": [(0, 1 << 20, np.int32), (0, 1 << 40, np.int64)],
             "wide": [(np.iinfo(np.int64).min, np.iinfo(np.int64).max, np.int64)] * 2}
    out = {"rows": n, "repeats": repeats}
    for name, spec in specs.items():
        log("composite keys: %s, n = %d" % (name, n))
        rc = [rng.integers(lo, hi, n, dtype=np.int64).astype(dt) for lo, hi, dt in spec]
        sc = [rng.integers(lo, hi, n, dtype=np.int64).astype(dt) for lo, hi, dt in spec]
        m = int(0.8 * n)
        idx = rng.integers(0, n, m)
        for a, b in zip(rc, sc):
            b[:m] = a[idx]
        drc = [torch.from_numpy(c).to("cuda") for c in rc]
        dsc = [torch.from_numpy(c).to("cuda") for c in sc]
        del rc, sc
        rid = torch.arange(n, dtype=torch.int32, device="cuda")
        res = {}
        for op in ("sort", "join"):
            times = []
            for i in range(repeats + 1):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if op == "sort":
                    outs, rout, st = tj.sort_multi(drc, rid, stats=True)
                else:
                    pr, ps, st = tj.join_multi(drc, rid, dsc, rid, stats=True)
                torch.cuda.synchronize()
                if i:
                    times.append((time.perf_counter() - t0) * 1e3)
            if op == "sort":
                k0, k1 = outs
                ok = bool(((k0[1:] > k0[:-1]) | ((k0[1:] == k0[:-1]) & (k1[1:] >= k1[:-1]))).all().item())
                assert ok, "composite sort output not ordered"
                res["sort"] = {"ms": round(pct(times, 0.5), 3), "rows_per_s": round(n / (pct(times, 0.5) * 1e-3), 1),
                               "sort_passes": st["passes"]}
                del outs, rout
            else:
                ok = all(torch.equal(a[pr.long()], b[ps.long()]) for a, b in zip(drc, dsc))
                assert ok, "composite join pairs do not match"
                res["join"] = {"ms": round(pct(times, 0.5), 3), "pairs": int(pr.numel()),
                               "tuples_per_s": round(2 * n / (pct(times, 0.5) * 1e-3), 1),
                               "note": "count, then materialise (two calls)"}
                del pr, ps
        out[name] = res
        del drc, dsc, rid
        torch.cuda.empty_cache()
    return out


def path_selection(tj, torch, d_rk, d_sk_join, d_sort, join_count: int, repeats: int = 5):
    """tj_select_path on the step's own inputs (the join's R and S, the sort
    column): HIP-event time of the sketch pass against its algorithmic bytes
    (every key read once), the indicators against the exact figures, and the
    decision; then the tensor path's join latency over a size sweep with the
    decision the default thresholds take at each size."""
    out = {}
    n_r, n_s = d_rk.numel(), d_sk_join.numel()
    ws = torch.empty(tj.select_workspace_query(max(n_r, d_sort.numel()), n_s), dtype=torch.uint8, device="cuda")
    for name, args, nbytes in (("join", (d_rk, d_sk_join), 8 * (n_r + n_s)), ("sort", (d_sort,), 8 * d_sort.numel())):
        ms = []
        for i in range(repeats + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            sel = tj.select_path(*args, workspace=ws)
            b.record()
            b.synchronize()
            if i:
                ms.append(a.elapsed_time(b))
        t = pct(ms, 0.5)
        rec = {"ms": round(t, 4), "bytes": nbytes, "GBs": round(nbytes / (t * 1e-3) / 1e9, 1),
               "hbm_frac": round(nbytes / (t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "path": "tensor" if sel["path"] else "linear", "reasons": sel["reasons"],
               "distinct_r": round(sel["distinct_r"], 1)}
        if name == "join":
            rec.update({"distinct_s": round(sel["distinct_s"], 1), "distinct_common": round(sel["distinct_common"], 1),
                        "est_output": round(sel["est_output"], 1), "exact_output": join_count,
                        "exact_distinct_r": n_r})
        out[name] = rec
        log("path selection %s: %.3f ms, %s" % (name, t, rec["path"]))
    del ws
    sweep = []
    import tjgen
    for lg in CROSSOVER_LOGS:
        w = tjgen.crossover(lg)
        r, s = torch.from_numpy(w["r_keys"]).to("cuda"), torch.from_numpy(w["s_keys"]).to("cuda")
        rr, sr = torch.from_numpy(w["r_rids"]).to("cuda"), torch.from_numpy(w["s_rids"]).to("cuda")
        sel_ms, join_ms, sort_ms = [], [], []
        for i in range(11):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sel = tj.select_path(r, s)
            t1 = time.perf_counter()
            pr, _ = tj.join(r, rr, s, sr)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tj.sort(s, sr)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            if i:
                sel_ms.append((t1 - t0) * 1e3)
                join_ms.append((t2 - t1) * 1e3)
                sort_ms.append((t3 - t2) * 1e3)
        assert pr.numel() == w.expected_count
        sweep.append({"rows_per_side": 1 << lg, "select_ms": round(pct(sel_ms, 0.5), 4),
                      "join_ms": round(pct(join_ms, 0.5), 4), "sort_ms": round(pct(sort_ms, 0.5), 4),
                      "pairs": int(pr.numel()), "est_output": round(sel["est_output"], 1),
                      "path": "tensor" if sel["path"] else "linear", "reasons": sel["reasons"]})
    out["sweep"] = sweep
    out["thresholds"] = {"min_rows": tj.TJ_SELECT_DEFAULT_MIN_ROWS, "min_output": tj.TJ_SELECT_DEFAULT_MIN_OUTPUT}
    return out


CROSSOVER_LOGS = tuple(range(8, 23, 2))


def stream_copy(tj, torch, mib: int = 4096, repeats: int = 10):
    """Bandwidth of the hand-written streaming copy and of torch's copy_ on the
    same buffers (HIP events on the current stream, median of `repeats`)."""
    nb = mib << 20
    src = torch.ones(nb // 8, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    out = {"bytes_copied": nb}
    for name, f in (("hand_written", lambda: tj.debug_stream_copy(src, dst)), ("torch_copy", lambda: dst.copy_(src))):
        ms = []
        for i in range(repeats + 2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            f()
            b.record()
            b.synchronize()
            if i >= 2:
                ms.append(a.elapsed_time(b))
        t = pct(ms, 0.5)
        gbs = 2 * nb / (t * 1e-3) / 1e9
        out[name] = {"ms": round(t, 4), "GBs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4)}
    assert torch.equal(src[:1 << 20], dst[:1 << 20]), "copy wrong"
    out["achievable_GBs"] = max(out["hand_written"]["GBs"], out["torch_copy"]["GBs"])
    log("stream copy: %.1f GB/s hand-written, %.1f GB/s torch" % (out["hand_written"]["GBs"],
                                                                  out["torch_copy"]["GBs"]))
    del src, dst
    torch.cuda.empty_cache()
    return out


def c1_small(tj, torch, repeats: int = 100, warmup: int = 10):
    """GPU P50/P99 (wall clock, synchronised) of the sort of R and the join of
    R and S at |R| = |S| = 10^5 int32 keys uniform in [0, 2^20)."""
    import tjgen
    w = tjgen.small_uniform()
    d = {k: torch.from_numpy(v).to("cuda") for k, v in w.items()}
    count = tj.join_count(d["r_keys"], d["s_keys"])
    out_r = torch.empty(max(count, 1), dtype=torch.int32, device="cuda")
    out_s = torch.empty_like(out_r)
    ko, ro = torch.empty_like(d["r_keys"]), torch.empty_like(d["r_rids"])
    ws_s = torch.empty(tj.workspace_query(tj.TJ_OP_SORT, tj.TJ_KEY_I32, 10 ** 5)[1], dtype=torch.uint8,
                       device="cuda")
    ws_j = torch.empty(tj.workspace_query(tj.TJ_OP_JOIN_MATERIALIZE, tj.TJ_KEY_I32, 10 ** 5, 10 ** 5)[1],
                       dtype=torch.uint8, device="cuda")
    ops = {"sort": lambda: tj.sort(d["r_keys"], d["r_rids"], keys_out=ko, rids_out=ro, workspace=ws_s),
           "join": lambda: tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=count,
                                   out_r=out_r, out_s=out_s, workspace=ws_j)}
    res = {"rows_per_side": 10 ** 5, "join_count": count, "repeats": repeats}
    for op, f in ops.items():
        times = []
        with no_gc():
            for i in range(warmup + repeats):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f()
                torch.cuda.synchronize()
                if i >= warmup:
                    times.append((time.perf_counter() - t0) * 1e3)
        # kernel time of one call (HIP events of every launch), in separate
        # calls so that the event records do not shift the latency above
        tj.timing(True)
        for _ in range(10):
            f()
        torch.cuda.synchronize()
        tj.timing(False)
        kms = sum(v["ms"] for k, v in tj.timing_read().items() if not k.startswith("host_")) / 10
        res[op] = {"p50_ms": round(pct(times, 0.5), 4), "p99_ms": round(pct(times, 0.99), 4),
                   "kernel_ms": round(kms, 4), "host_and_sync_ms": round(pct(times, 0.5) - kms, 4)}
    log("C1: sort P50 %.3f ms, join P50 %.3f ms" % (res["sort"]["p50_ms"], res["join"]["p50_ms"]))
    del d, out_r, out_s, ko, ro, ws_s, ws_j
    return res


def hbm_variants(tj, torch, steps: int):
    """The Zipf(0.99) HBM-scale join (R: 2^27 rows, the 2^20 hottest keys 4
    times; S: 2^29 rows, 80% matched by Zipf(0.99)) with a sort of its S keys,
    timed like the step; then the standalone sort of 2^29 keys uniform over
    [0, 2^40)."""
    import tjgen
    log("hbm zipf: generating")
    w = tjgen.hbm_scale(0.99)
    n_r, n_s = w["r_keys"].size, w["s_keys"].size
    d_rk = torch.from_numpy(w["r_keys"]).to("cuda")
    d_rr = torch.from_numpy(w["r_rids"]).to("cuda")
    d_sk = torch.from_numpy(w["s_keys"]).to("cuda")
    d_sr = torch.from_numpy(w["s_rids"]).to("cuda")
    expected = w.expected_count
    del w
    cap = 4 * n_s
    out_r = torch.empty(cap, dtype=torch.int32, device="cuda")
    out_s = torch.empty(cap, dtype=torch.int32, device="cuda")
    ko, ro = torch.empty_like(d_sk), torch.empty_like(d_sr)
    ws_sort = torch.empty(tj.workspace_query(tj.TJ_OP_SORT, tj.TJ_KEY_I64, n_s)[1], dtype=torch.uint8, device="cuda")
    ws_join = torch.empty(tj.workspace_query(tj.TJ_OP_JOIN_MATERIALIZE, tj.TJ_KEY_I64, n_r, n_s)[1],
                          dtype=torch.uint8, device="cuda")

    def sort():
        return tj.sort(d_sk, d_sr, keys_out=ko, rids_out=ro, workspace=ws_sort, stats=True)[2]

    def join():
        pr, _, st = tj.join(d_rk, d_rr, d_sk, d_sr, capacity=cap, out_r=out_r, out_s=out_s, workspace=ws_join,
                            stats=True)
        return pr.numel(), st

    sort()
    join()
    torch.cuda.synchronize()
    tj.timing(True)
    t_sort, t_join = [], []
    with no_gc():
        for i in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sts = sort()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            cnt, stj = join()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            t_sort.append(t1 - t0)
            t_join.append(t2 - t1)
            log("hbm zipf step %d: sort %.2f ms, join %.2f ms" % (i, (t1 - t0) * 1e3, (t2 - t1) * 1e3))
    tj.timing(False)
    fams = tj.timing_read()
    assert cnt == expected, "zipf join count %d != closed form %d" % (cnt, expected)
    assert bool((ko[1:] >= ko[:-1]).all().item()), "zipf sort output not ordered"
    step_s = (sum(t_sort) + sum(t_join)) / steps
    dom = max((f for f in fams if not f.startswith("host_")), key=lambda f: fams[f]["ms"])
    fd = fams[dom]
    avg_ms = fd["ms"] / max(fd["launches"], 1)
    bpl = fd["bytes"] / max(fd["launches"], 1)
    ach = bpl / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    planned = sts["bytes_read"] + sts["bytes_written"] + stj["bytes_read"] + stj["bytes_written"]
    zipf = {"workload": "hbm_scale theta=0.99: join |R|=2^27 x |S|=2^29 int64 keys (2^20 hottest R keys x4, "
                        "S 80%% matched by Zipf(0.99)) + sort of the 2^29 S keys; int32 row ids",
            "steps": steps, "join_count": cnt, "pair_capacity": cap,
            "tuples_per_s": round((2 * n_s + n_r) / step_s, 1),
            "sort_ms_p50": round(pct(t_sort, 0.5) * 1e3, 3), "sort_ms_max": round(max(t_sort) * 1e3, 3),
            "join_ms_p50": round(pct(t_join, 0.5) * 1e3, 3), "join_ms_max": round(max(t_join) * 1e3, 3),
            "pairs_per_s": round(cnt / pct(t_join, 0.5), 1),
            "planned_hbm_frac": round(planned / step_s / (HBM_PEAK_GBS * 1e9), 4),
            "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "bytes_per_launch": int(bpl),
                         "avg_launch_ms": round(avg_ms, 4), "launches_per_step": fd["launches"] / steps},
            "kernels": {f: {"launches_per_step": v["launches"] / steps, "ms_per_step": round(v["ms"] / steps, 3),
                            "GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
                        for f, v in fams.items() if v["launches"]},
            "plan": {"sort": sts, "join": stj}}
    log("hbm zipf: sort %.2f ms, join %.2f ms (%d pairs), %s %.1f GB/s" %
        (zipf["sort_ms_p50"], zipf["join_ms_p50"], cnt, dom, ach))
    del d_rk, d_rr, d_sk, d_sr, out_r, out_s, ko, ro, ws_sort, ws_join
    torch.cuda.empty_cache()
    # standalone sort, keys uniform over [0, 2^40)
    keys = torch.from_numpy(tjgen.sort_uniform64(1 << 29, bits=40)["keys"]).to("cuda")
    rids = torch.arange(keys.numel(), dtype=torch.int32, device="cuda")
    ko, ro = torch.empty_like(keys), torch.empty_like(rids)
    ws = torch.empty(tj.workspace_query(tj.TJ_OP_SORT, tj.TJ_KEY_I64, keys.numel())[1], dtype=torch.uint8,
                     device="cuda")
    times = []
    for i in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, st = tj.sort(keys, rids, keys_out=ko, rids_out=ro, workspace=ws, stats=True)
        torch.cuda.synchronize()
        if i:
            times.append(time.perf_counter() - t0)
    assert bool((ko[1:] >= ko[:-1]).all().item()), "40-bit sort output not ordered"
    s40 = {"workload": "sort of 2^29 int64 keys uniform over [0, 2^40), int32 row ids",
           "ms_p50": round(pct(times, 0.5) * 1e3, 3), "ms_max": round(max(times) * 1e3, 3),
           "keys_per_s": round(keys.numel() / pct(times, 0.5), 1), "passes": st["passes"]}
    log("sort 40-bit: %.2f ms" % s40["ms_p50"])
    del keys, rids, ko, ro, ws
    torch.cuda.empty_cache()
    return {"zipf_0.99": zipf, "sort_40bit": s40}


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_latencies(c2_repeats: int = 10):
    """The oracle built -O3 -march=native on this host, pinned to one core:
    C1 and paper-shaped P50/P99, and the size sweep's sort and join times."""
    import tempfile
    import oracle
    import tjgen
    tmp = tempfile.mkdtemp(prefix="tj_oracle_")
    orc = oracle.Oracle(oracle.build_native(tmp))
    before = os.sched_getaffinity(0)
    core = min(before)
    os.sched_setaffinity(0, {core})
    try:
        out = {"build": "g++ -O3 -march=native", "pinned_core": core, "threads": 1, "host": _host_cpu()}

        def lat(f, repeats, warm=1):
            ts = []
            for i in range(warm + repeats):
                t0 = time.perf_counter()
                f()
                if i >= warm:
                    ts.append((time.perf_counter() - t0) * 1e3)
            return {"p50_ms": round(pct(ts, 0.5), 4), "p99_ms": round(pct(ts, 0.99), 4), "repeats": repeats}

        w = tjgen.small_uniform()
        out["c1_small"] = {"sort": lat(lambda: orc.sort(w["r_keys"], w["r_rids"]), 100, 10),
                           "join": lat(lambda: orc.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"]),
                                       100, 10)}
        log("cpu C1 done")
        for theta in (0.0, 0.99):
            w = tjgen.paper_shaped(theta)
            out["paper_shaped_theta%g" % theta] = {
                "sort": lat(lambda: orc.sort(w["s_keys"], w["s_rids"]), c2_repeats),
                "join": lat(lambda: orc.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"]), c2_repeats)}
            log("cpu paper-shaped theta %g done" % theta)
        sweep = []
        for lg in CROSSOVER_LOGS:
            w = tjgen.crossover(lg)
            reps = 20 if lg <= 16 else (3 if lg <= 18 else 1)
            sweep.append({"rows_per_side": 1 << lg,
                          "sort_ms": lat(lambda: orc.sort(w["s_keys"], w["s_rids"]), reps)["p50_ms"],
                          "join_ms": lat(lambda: orc.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"],
                                                                w["s_rids"]), reps)["p50_ms"]})
        out["sweep"] = sweep
        log("cpu sweep done")
    finally:
        os.sched_setaffinity(0, before)
    return out


def crossover(gpu_sweep, cpu_sweep, key):
    """Smallest size (rows per side, interpolated on log2 size between the two
    measured sizes around it) from which the tensor path's time stays below the
    oracle's; None when it never does."""
    pts = [(np.log2(g["rows_per_side"]), g[key] - c[key]) for g, c in zip(gpu_sweep, cpu_sweep)]
    last = None
    for i in range(len(pts)):
        if all(d < 0 for _, d in pts[i:]):
            last = i
            break
    if last is None:
        return None
    if last == 0:
        return {"rows_per_side": int(2 ** pts[0][0]), "below_sweep": True}
    (x0, d0), (x1, d1) = pts[last - 1], pts[last]
    x = x0 + (x1 - x0) * d0 / (d0 - d1)
    return {"rows_per_side": int(round(2 ** x)), "below_sweep": False}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="hbm", choices=["hbm", "paper", "small"])
    ap.add_argument("--theta", type=float, default=0.0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-sweep", action="store_true", help="skip the paper-shaped budget sweep")
    ap.add_argument("--sweep-repeats", type=int, default=100)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-vs-radix comparison")
    ap.add_argument("--learned-rows", type=int, default=1 << 28,
                    help="rows per relation of the learned-vs-radix comparison")
    ap.add_argument("--learned-repeats", type=int, default=5)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-loop measurement")
    ap.add_argument("--no-multi", action="store_true", help="skip the composite-key measurement")
    ap.add_argument("--no-select", action="store_true", help="skip the path-selection measurement")
    ap.add_argument("--multi-rows", type=int, default=1 << 26)
    ap.add_argument("--serve-requests", type=int, default=1000, help="arrivals per rate")
    ap.add_argument("--serve-rates", default="50,200,800,3200", help="arrival rates, requests/s")
    ap.add_argument("--serve-pool", type=int, default=64, help="requests resident on the device")
    ap.add_argument("--only-serving", action="store_true",
                    help="run the serving measurement alone (no step, no other section) and print its JSON")
    ap.add_argument("--no-copy", action="store_true", help="skip the streaming-copy bandwidth line")
    ap.add_argument("--no-c1", action="store_true", help="skip the small (10^5-row) latency line")
    ap.add_argument("--no-zipf", action="store_true", help="skip the Zipf(0.99) HBM-scale section")
    ap.add_argument("--zipf-steps", type=int, default=5)
    ap.add_argument("--c2-repeats", type=int, default=10, help="oracle repeats of the paper-shaped workload")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="before timing, copy MIB MiB device-to-device three times (a plain copy "
                         "of known size that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sort and join run on a single MI355X "
              "(multi-GPU key-range sharding is a design note, not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2602_21237_amd as tj

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tj.load()
    if args.only_serving:
        res = serving(tj, torch, [float(r) for r in args.serve_rates.split(",")], args.serve_requests,
                      pool=args.serve_pool)
        print(json.dumps({"serving": res}), flush=True)
        return
    log("generating workload %s" % args.workload)
    w, sort_keys, desc = make_workload(args.workload, args.theta)
    kt = tj.TJ_KEY_I64 if sort_keys.dtype == np.int64 else tj.TJ_KEY_I32
    n_sort, n_r, n_s = sort_keys.size, w["r_keys"].size, w["s_keys"].size
    d_sk = torch.from_numpy(sort_keys).to("cuda")
    d_sr = torch.arange(n_sort, dtype=torch.int32, device="cuda")
    d_rk = torch.from_numpy(w["r_keys"]).to("cuda")
    d_rr = torch.from_numpy(w["r_rids"]).to("cuda")
    d_skj = torch.from_numpy(w["s_keys"]).to("cuda")
    d_srj = torch.from_numpy(w["s_rids"]).to("cuda")
    expected = w.expected_count
    del sort_keys
    cap = 4 * n_s if args.workload == "hbm" else (expected if expected is not None else 4 * n_s)
    ko, ro = torch.empty_like(d_sk), torch.empty_like(d_sr)
    out_r = torch.empty(cap, dtype=torch.int32, device="cuda")
    out_s = torch.empty(cap, dtype=torch.int32, device="cuda")
    ws_sort = torch.empty(tj.workspace_query(tj.TJ_OP_SORT, kt, n_sort)[1], dtype=torch.uint8, device="cuda")
    ws_join = torch.empty(tj.workspace_query(tj.TJ_OP_JOIN_MATERIALIZE, kt, n_r, n_s)[1],
                          dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    log("inputs resident: sort %d rows, join %d x %d rows" % (n_sort, n_r, n_s))

    def step():
        _, _, st_sort = tj.sort(d_sk, d_sr, keys_out=ko, rids_out=ro, workspace=ws_sort, stats=True)
        pr, _, st_join = tj.join(d_rk, d_rr, d_skj, d_srj, capacity=cap, out_r=out_r, out_s=out_s,
                                 workspace=ws_join, stats=True)
        return pr.numel(), st_sort, st_join

    for i in range(args.warmup):
        cnt, _, _ = step()
        log("warmup %d done, join count %d" % (i, cnt))

    if args.copy_calibration > 0:
        nb = args.copy_calibration << 20
        c_src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        c_dst = torch.empty_like(c_src)
        for _ in range(3):
            c_dst.copy_(c_src)
        torch.cuda.synchronize()
        log("copy calibration: %d bytes copied 3 times" % nb)
        del c_src, c_dst

    tj.timing(True)
    torch.cuda.synchronize()
    times, t_sort, t_join = [], [], []
    with no_gc():
        for i in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, sts = tj.sort(d_sk, d_sr, keys_out=ko, rids_out=ro, workspace=ws_sort, stats=True)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            pr, _, stj = tj.join(d_rk, d_rr, d_skj, d_srj, capacity=cap, out_r=out_r, out_s=out_s,
                                 workspace=ws_join, stats=True)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append(t2 - t0)
            t_sort.append(t1 - t0)
            t_join.append(t2 - t1)
            log("step %d: sort %.2f ms, join %.2f ms" % (i, (t1 - t0) * 1e3, (t2 - t1) * 1e3))
    tj.timing(False)
    fams = tj.timing_read()
    # properties of the last step's results that hold at any size
    if expected is not None:
        assert pr.numel() == expected, "join count %d != closed form %d" % (pr.numel(), expected)
    assert bool((ko[1:] >= ko[:-1]).all().item()), "sort output not ordered"
    total_s = sum(times)
    ms_per_step = total_s / args.steps * 1e3
    tuples = n_sort + n_r + n_s
    value = tuples / (total_s / args.steps)

    dom = max((f for f in fams if not f.startswith("host_")), key=lambda f: fams[f]["ms"])
    fd = fams[dom]
    avg_ms = fd["ms"] / max(fd["launches"], 1)
    bytes_per_launch = fd["bytes"] / max(fd["launches"], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic, traffic_src = measured_traffic(dom, args.workload + ("_theta%g" % args.theta if args.theta else ""))
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": traffic_src, "kernel_source_sha256_16": kernel_source_digest(),
                "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_ms, 4),
                "launches_per_step": fd["launches"] / args.steps}
    kernels = {f: {"launches_per_step": v["launches"] / args.steps,
                   "ms_per_step": round(v["ms"] / args.steps, 3),
                   "GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
               for f, v in fams.items() if v["launches"]}
    planned = sts["bytes_read"] + sts["bytes_written"] + stj["bytes_read"] + stj["bytes_written"]
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "tuples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64" if kt == 8 else "int32",
        "data": "synthetic (seeded generators; no dataset)",
        "config": {"workload": desc, "sort_rows": n_sort, "n_r": n_r, "n_s": n_s,
                   "join_count": int(pr.numel()), "pair_capacity": cap, "parallelism": "single GPU"},
        "sort_keys_per_s": round(n_sort / (sum(t_sort) / args.steps), 1),
        "join_tuples_per_s": round((n_r + n_s) / (sum(t_join) / args.steps), 1),
        "p50_step_ms": round(pct(times, 0.5) * 1e3, 3), "p99_step_ms": round(pct(times, 0.99) * 1e3, 3),
        "host_and_sync_ms_per_step": round(ms_per_step - sum(v["ms"] for f, v in fams.items()
                                                             if not f.startswith("host_")) / args.steps, 3),
        "planned_hbm_frac": round(planned / (ms_per_step * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
        "roofline": roofline, "kernels": kernels,
        "plan": {"sort": sts, "join": stj},
    }
    if not args.no_select:
        line["path_selection"] = path_selection(tj, torch, d_rk, d_skj, d_sk, int(pr.numel()))
    del ko, ro, out_r, out_s, ws_sort, ws_join, d_sk, d_sr, d_rk, d_rr, d_skj, d_srj
    torch.cuda.empty_cache()
    if not args.no_copy:
        line["stream_copy"] = stream_copy(tj, torch)
        line["roofline"]["achievable_GBs"] = line["stream_copy"]["achievable_GBs"]
        line["roofline"]["frac_of_achievable"] = round(achieved / line["stream_copy"]["achievable_GBs"], 4)
    if not args.no_c1:
        line["c1_small"] = c1_small(tj, torch)
    if not args.no_zipf and args.workload == "hbm":
        line["hbm_zipf"] = hbm_variants(tj, torch, args.zipf_steps)
    if not args.no_learned:
        line["learned_vs_radix"] = learned_vs_radix(tj, torch, args.learned_rows, args.learned_repeats)
    if not args.no_multi:
        line["composite_keys"] = composite_keys(tj, torch, args.multi_rows)
    if not args.no_serving:
        line["serving"] = serving(tj, torch, [float(r) for r in args.serve_rates.split(",")], args.serve_requests,
                                  pool=args.serve_pool)
    if not args.no_sweep:
        log("paper-shaped budget sweep")
        line["paper_shaped"] = paper_shaped_sweep(tj, torch, args.sweep_repeats)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(args.workload, args.theta)
        lat = cpu_latencies(args.c2_repeats)
        line["cpu_baseline"]["native_pinned"] = lat
        if "path_selection" in line:
            ps = line["path_selection"]
            ps["oracle_sweep"] = lat["sweep"]
            ps["crossover"] = {"join": crossover(ps["sweep"], lat["sweep"], "join_ms"),
                               "sort": crossover(ps["sweep"], lat["sweep"], "sort_ms")}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""The memory contract of the C ABI, checked with guard regions.

Every output column and the workspace are sub-views of larger buffers whose
remaining bytes (1 MiB after each region, and 1 MiB before the workspace)
hold a pattern. After sorts, counts and materialisations at the three budget
regimes (the minimum workspace, 1 MiB, the full workspace), a capacity
overflow and the learned pass, the pattern must be untouched: no call writes
at or beyond `capacity` / `n` / `workspace_bytes`, or before the workspace.
Outputs are also compared with the oracle, and once the kernels are loaded the
device's free memory must not change across calls (the library allocates
nothing).
"""
import numpy as np
import pytest

import oracle
import tjgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

G = 1 << 20  # guard bytes
PAT = 0xA5


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


class Guarded:
    """A device region of `nbytes` bytes (viewed as `dtype`) with G pattern
    bytes after it, and optionally G before it."""

    def __init__(self, nbytes, dtype=torch.uint8, before=False):
        self.pre = G if before else 0
        self.nbytes = nbytes
        self.buf = torch.full((self.pre + nbytes + G,), PAT, dtype=torch.uint8, device="cuda")
        raw = self.buf[self.pre:self.pre + nbytes]
        self.view = raw.view(dtype) if nbytes else torch.empty(0, dtype=dtype, device="cuda")

    def intact(self):
        tail = self.buf[self.pre + self.nbytes:]
        ok = bool((tail == PAT).all().item())
        if self.pre:
            ok = ok and bool((self.buf[:self.pre] == PAT).all().item())
        return ok


def _ws(tj, op, kt, n_r, n_s, budget):
    mn, full = tj.workspace_query(op, kt, n_r, n_s)
    b = {"min": mn, "1MiB": max(mn, 1 << 20), "full": full}[budget]
    return Guarded(b, before=True), b


@pytest.fixture(scope="module")
def work():
    w = tjgen.paper_shaped(0.99, n=1_000_000, rid_perm=True)
    d = {k: torch.from_numpy(v).to("cuda") for k, v in w.items()}
    ek, er = oracle.sort(w["s_keys"], w["s_rids"])
    xr, xs, cnt = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    return w, d, (ek, er), (xr, xs, cnt)


@pytest.mark.parametrize("budget", ["min", "1MiB", "full"])
def test_sort_guards(tj, work, budget):
    w, d, (ek, er), _ = work
    n = d["s_keys"].numel()
    ws, b = _ws(tj, tj.TJ_OP_SORT, tj.TJ_KEY_I64, n, 0, budget)
    ko, ro = Guarded(n * 8, torch.int64), Guarded(n * 4, torch.int32)
    tj.sort(d["s_keys"], d["s_rids"], keys_out=ko.view, rids_out=ro.view, workspace=ws.view, workspace_bytes=b)
    torch.cuda.synchronize()
    assert ko.intact() and ro.intact() and ws.intact(), "a guard region was written"
    assert np.array_equal(ko.view.cpu().numpy(), ek) and np.array_equal(ro.view.cpu().numpy(), er)


@pytest.mark.parametrize("budget", ["min", "1MiB", "full"])
def test_join_guards(tj, work, budget):
    w, d, _, (xr, xs, cnt) = work
    nr, ns = d["r_keys"].numel(), d["s_keys"].numel()
    ws, b = _ws(tj, tj.TJ_OP_JOIN_MATERIALIZE, tj.TJ_KEY_I64, nr, ns, budget)
    c = tj.join_count(d["r_keys"], d["s_keys"], workspace=ws.view, workspace_bytes=b)
    assert c == cnt and ws.intact()
    o_r, o_s = Guarded(cnt * 4, torch.int32), Guarded(cnt * 4, torch.int32)
    pr, ps = tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=cnt, out_r=o_r.view,
                     out_s=o_s.view, workspace=ws.view, workspace_bytes=b)
    torch.cuda.synchronize()
    assert o_r.intact() and o_s.intact() and ws.intact(), "a guard region was written"
    assert np.array_equal(pr.cpu().numpy(), xr) and np.array_equal(ps.cpu().numpy(), xs)
    # capacity one short: TJ_E_CAPACITY, the count set, nothing written at or beyond capacity
    cap = cnt - 1
    o_r2, o_s2 = Guarded(cap * 4, torch.int32), Guarded(cap * 4, torch.int32)
    with pytest.raises(tj.TjError) as ei:
        tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=cap, out_r=o_r2.view,
                out_s=o_s2.view, workspace=ws.view, workspace_bytes=b)
    assert ei.value.status == -3
    torch.cuda.synchronize()
    assert o_r2.intact() and o_s2.intact() and ws.intact(), "written at or beyond capacity"


def test_learned_guards(tj):
    w = tjgen.learned("lognormal", 400_003)
    d = {k: torch.from_numpy(v).to("cuda") for k, v in w.items()}
    n = d["r_keys"].numel()
    ws, b = _ws(tj, tj.TJ_OP_SORT, tj.TJ_KEY_I64, n, 0, "full")
    ko, ro = Guarded(n * 8, torch.int64), Guarded(n * 4, torch.int32)
    _, _, st = tj.sort(d["r_keys"], d["r_rids"], keys_out=ko.view, rids_out=ro.view, workspace=ws.view,
                       workspace_bytes=b, stats=True, partitioner="learned", learned_min_rows=1)
    torch.cuda.synchronize()
    assert st["learned"] == 1 and ko.intact() and ro.intact() and ws.intact()
    ek, er = oracle.sort(w["r_keys"], w["r_rids"])
    assert np.array_equal(ko.view.cpu().numpy(), ek) and np.array_equal(ro.view.cpu().numpy(), er)
    xr, xs, cnt = oracle.join_pairs(w["r_keys"], w["r_rids"], w["s_keys"], w["s_rids"])
    wsj, bj = _ws(tj, tj.TJ_OP_JOIN_MATERIALIZE, tj.TJ_KEY_I64, n, d["s_keys"].numel(), "full")
    o_r, o_s = Guarded(cnt * 4, torch.int32), Guarded(cnt * 4, torch.int32)
    pr, ps, st = tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=cnt, out_r=o_r.view,
                         out_s=o_s.view, workspace=wsj.view, workspace_bytes=bj, stats=True,
                         partitioner="learned", learned_min_rows=1)
    torch.cuda.synchronize()
    assert st["learned"] == 1 and o_r.intact() and o_s.intact() and wsj.intact()
    assert np.array_equal(pr.cpu().numpy(), xr) and np.array_equal(ps.cpu().numpy(), xs)


def test_calls_allocate_nothing(tj, work):
    """With the caller's outputs and workspace in place, a sequence of calls
    leaves the device's free memory exactly where it was."""
    w, d, _, (xr, xs, cnt) = work
    nr, ns = d["r_keys"].numel(), d["s_keys"].numel()
    _, full = tj.workspace_query(tj.TJ_OP_JOIN_MATERIALIZE, tj.TJ_KEY_I64, nr, ns)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    ko, ro = torch.empty_like(d["s_keys"]), torch.empty_like(d["s_rids"])
    o_r = torch.empty(cnt, dtype=torch.int32, device="cuda")
    o_s = torch.empty(cnt, dtype=torch.int32, device="cuda")
    def calls():
        tj.sort(d["s_keys"], d["s_rids"], keys_out=ko, rids_out=ro, workspace=ws)
        tj.join_count(d["r_keys"], d["s_keys"], workspace=ws)
        tj.join(d["r_keys"], d["r_rids"], d["s_keys"], d["s_rids"], capacity=cnt, out_r=o_r, out_s=o_s,
                workspace=ws)
        for b in (1 << 20, 64 << 20):
            tj.sort(d["s_keys"], d["s_rids"], keys_out=ko, rids_out=ro, workspace=ws, workspace_bytes=b)
            tj.join_count(d["r_keys"], d["s_keys"], workspace=ws, workspace_bytes=b)

    # The first round loads the kernels' code (and the runtime's per-kernel
    # scratch backing); the rounds after it must not change free memory.
    calls()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(2):
        calls()
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert np.array_equal(o_r.cpu().numpy(), xr) and np.array_equal(o_s.cpu().numpy(), xs)

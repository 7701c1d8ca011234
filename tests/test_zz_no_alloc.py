"""tj_sort_static (the sort on the library's own device scratch) against
tj_sort with a caller workspace: bit-exact outputs on two calls in a row, the
second with a smaller input, plus the oracle on a sample of positions; the
call leaves the device's free memory unchanged.

The first call is larger than the scratch's unlimited plan (beyond 22,346,560
int64 or 33,519,872 int32 rows), so it runs the budget-bound plan (its output
columns plus a window of the scratch); the second fits the unlimited plan.
"""
import numpy as np
import pytest

import oracle
import tjgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    # The first call on a device loads the scratch's code object (and with it
    # the array) and looks up its address; free memory is compared after it.
    k = torch.arange(16, dtype=torch.int64, device="cuda")
    r = torch.arange(16, dtype=torch.int32, device="cuda")
    p.sort_static(k, r, torch.empty_like(k), torch.empty_like(r))
    torch.cuda.synchronize()
    return p


def _case(n, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "i64":
        k = rng.integers(-(1 << 62), 1 << 62, n, dtype=np.int64)
        k[rng.integers(0, n, n // 8)] = k[rng.integers(0, n, n // 8)]  # duplicated keys
    else:
        k = rng.integers(-(1 << 20), 1 << 20, n, dtype=np.int64).astype(np.int32)
    r = tjgen.perm_i32(n, seed)
    return k, r


@pytest.mark.parametrize("kind,n1,n2", [("i64", 3 << 23, (1 << 20) + 7), ("i32", 40_000_001, 4097)])
def test_static_sort_equals_tj_sort(tj, kind, n1, n2):
    for call, n in enumerate((n1, n2)):
        print("tj_sort_static case %s call %d n=%d" % (kind, call, n), flush=True)
        k, r = _case(n, kind, 11 + call)
        dk, dr = torch.from_numpy(k).cuda(), torch.from_numpy(r).cuda()
        ek, er, st_ref = tj.sort(dk, dr, stats=True)
        ko = torch.full_like(dk, 0x5A5A5A5A)
        ro = torch.full_like(dr, 0x5A5A5A5A)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        st = tj.sort_static(dk, dr, ko, ro, stats=True)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0, "free device memory changed across the call: %d -> %d" % (free0, free1)
        assert torch.equal(ko, ek) and torch.equal(ro, er), "tj_sort_static differs from tj_sort"
        if call == 0:
            assert st["key_ranges"] > 1 or st["windows"] > 0, st  # the budget binds inside the scratch
        else:
            assert st["key_ranges"] == 1 and st["windows"] == 0, st
        # a sample of positions against the oracle (the full oracle sort is slow at 2.5e7 rows)
        xk, xr = oracle.sort(k, r) if n <= (1 << 21) else (None, None)
        if xk is not None:
            assert np.array_equal(ko.cpu().numpy(), xk) and np.array_equal(ro.cpu().numpy(), xr)
        del dk, dr, ko, ro, ek, er
        torch.cuda.empty_cache()


def test_static_sort_empty_and_errors(tj):
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    er = torch.empty(0, dtype=torch.int32, device="cuda")
    assert tj.sort_static(e, er, e.clone(), er.clone(), stats=True)["leaves"] == 0
    k = torch.arange(10, dtype=torch.int64, device="cuda")
    r = torch.arange(10, dtype=torch.int32, device="cuda")
    with pytest.raises(tj.TjError) as ei:
        tj.sort_static(k, r, k, r.clone())  # output aliases the input
    assert ei.value.status == -5

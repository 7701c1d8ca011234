"""GPU parity of the execution-time path selection (tj_select_path).

The device sketch must hold the oracle's HyperLogLog registers bit for bit
(R, S and their union); the estimates are then the same float64 formula of
the same register counts on both sides, and the decision must agree. At the
benchmark's full join size the oracle's registers are computed too, and the
estimates are checked against the known distinct counts of the workload.
"""
import numpy as np
import pytest

import tjgen
from oracle import pathsel as S

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


def _check(tj, r, s=None, **kw):
    regs = torch.full((3 * S.M,), 0xAB, dtype=torch.uint8, device="cuda")
    got = tj.select_path(dev(r), None if s is None else dev(s), registers=regs, **kw)
    want = S.select(r, s, **kw)
    assert np.array_equal(regs.cpu().numpy().reshape(3, S.M), want["registers"])
    for f in ("distinct_r", "distinct_s", "distinct_union", "distinct_common", "est_output"):
        assert got[f] == pytest.approx(want[f], rel=1e-12, abs=1e-12), f
    for f in ("n_r", "n_s", "path", "reasons"):
        assert got[f] == want[f], f
    # the same call without a registers output gives the same selection
    again = tj.select_path(dev(r), None if s is None else dev(s), **kw)
    assert again == got
    return got


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("n", [0, 1, 1000, 4096, 3 * 16384 + 17, (1 << 20) + 13, 512 * 16384, 512 * 16384 + 1])
def test_sort_selection(tj, dtype, n):
    rng = np.random.default_rng(n + 1)
    info = np.iinfo(dtype)
    r = rng.integers(info.min, info.max, size=n, dtype=dtype)
    _check(tj, r)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("n_r,n_s", [(0, 0), (0, 5000), (777, 0), (5000, 123457), (300001, 1 << 21)])
def test_join_selection(tj, dtype, n_r, n_s):
    rng = np.random.default_rng(n_r * 7 + n_s)
    r = rng.integers(-(1 << 20), 1 << 20, size=n_r).astype(dtype)
    s = rng.integers(-(1 << 21), 1 << 20, size=n_s).astype(dtype)
    _check(tj, r, s)


@pytest.mark.parametrize("dtype,offset", [(np.int64, 1), (np.int64, 3), (np.int32, 1), (np.int32, 2), (np.int32, 3)])
def test_unaligned_columns(tj, dtype, offset):
    """Columns that do not start on a 16-byte boundary take the scalar-load
    kernel; the registers must not change."""
    rng = np.random.default_rng(offset)
    info = np.iinfo(dtype)
    full = rng.integers(info.min, info.max, size=300007 + offset, dtype=dtype)
    sfull = rng.integers(-1000, 1000, size=70001 + offset).astype(dtype)
    d, ds = dev(full)[offset:], dev(sfull)[offset:]
    assert d.data_ptr() % 16 != 0
    regs = torch.zeros(3 * S.M, dtype=torch.uint8, device="cuda")
    got = tj.select_path(d, ds, registers=regs)
    want = S.select(full[offset:], sfull[offset:])
    assert np.array_equal(regs.cpu().numpy().reshape(3, S.M), want["registers"])
    assert got["distinct_union"] == pytest.approx(want["distinct_union"], rel=1e-12)


def test_extreme_keys_and_duplicates(tj):
    ext = np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0, -1, 1], dtype=np.int64)
    r = np.repeat(ext, 40000)
    _check(tj, r, r[::-1].copy())
    r32 = np.array([np.iinfo(np.int32).min, np.iinfo(np.int32).max, 0, -1], dtype=np.int32)
    _check(tj, np.tile(r32, 5000))


@pytest.mark.parametrize("theta", [0.0, 0.99])
def test_paper_shaped(tj, theta):
    w = tjgen.paper_shaped(theta)
    got = _check(tj, w["r_keys"], w["s_keys"])
    assert got["path"] == 1
    # the exact output of the workload bounds what a uniform-spread estimate may say
    n = w["r_keys"].size
    assert abs(got["distinct_r"] - np.unique(w["r_keys"]).size) <= 0.03 * n


def test_thresholds(tj):
    rng = np.random.default_rng(5)
    many = rng.integers(0, 50, size=4000, dtype=np.int64)
    for mr, mo in ((0, 0), (10**9, 1), (10**9, 10**9), (8000, 10**9), (8001, 10**9)):
        _check(tj, many, many, min_rows=mr, min_output=mo)


def test_full_size_join(tj):
    """The benchmark's join inputs (2^27 R rows with distinct keys, 2^29 S
    rows): registers against the oracle's, estimates against the known
    distinct counts."""
    w = tjgen.hbm_scale(0.0)
    r, s = w["r_keys"], w["s_keys"]
    got = _check(tj, r, s)
    sigma = 1.04 / np.sqrt(S.M)
    assert abs(got["distinct_r"] - r.size) <= 3 * sigma * r.size  # R's keys are distinct
    assert got["path"] == 1 and got["reasons"] & 1


def test_side_stream_and_join_ops(tj):
    """The selection runs on the caller's stream, and both join ops give the
    same selection."""
    import ctypes
    from paper_2602_21237_amd import tj as tjm
    rng = np.random.default_rng(9)
    r = rng.integers(0, 1 << 30, size=200003, dtype=np.int64)
    s = rng.integers(0, 1 << 30, size=100001, dtype=np.int64)
    dr, ds = dev(r), dev(s)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = tj.select_path(dr, ds, stream=side)
    want = S.select(r, s)
    assert got["path"] == want["path"] and got["distinct_union"] == pytest.approx(want["distinct_union"], rel=1e-12)
    lib = tjm.load()
    need = tj.select_workspace_query(r.size, s.size)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = []
    for op in (tj.TJ_OP_JOIN_COUNT, tj.TJ_OP_JOIN_MATERIALIZE):
        o = tjm.Selection()
        assert lib.tj_select_path(op, 8, dr.data_ptr(), r.size, ds.data_ptr(), s.size, None, ctypes.byref(o), None,
                                  ws.data_ptr(), need, None) == 0
        outs.append(o.as_dict())
    assert outs[0] == outs[1] == got

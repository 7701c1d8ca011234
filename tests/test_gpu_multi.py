"""GPU parity of the composite-key sort and join against the composite-key
oracle: packed keys of 4 and 8 bytes, groups of columns sorted least
significant first when their widths exceed 64 bits, and the dense-rank join
beyond 64 bits."""
import numpy as np
import pytest

from oracle import multi

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
I64 = np.iinfo(np.int64)
I32 = np.iinfo(np.int32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def tj():
    import paper_2602_21237_amd as p
    p.load()
    return p


def _cols(rng, n, spec):
    out = []
    for lo, hi, dt in spec:
        out.append(rng.integers(lo, hi, n, dtype=np.int64, endpoint=False).astype(dt) if hi > lo
                   else np.full(n, lo, dtype=dt))
    return out


SPECS = {
    "packed32": [(-100, 100, np.int32), (0, 1000, np.int64)],               # 8 + 10 bits: 4-byte key
    "packed64": [(0, 1 << 30, np.int64), (-5, 5, np.int32), (0, 1 << 20, np.int32)],  # 30 + 4 + 20 bits
    "wide2": [(I64.min, I64.max, np.int64), (I64.min, I64.max, np.int64)],    # 128 bits: two groups
    "wide3": [(0, 4, np.int32), (I64.min, I64.max, np.int64), (I32.min, I32.max, np.int32)],
    "constant": [(7, 7, np.int64), (0, 3, np.int32), (-9, -9, np.int32)],
    "one": [(I64.min, I64.max, np.int64)],
}


@pytest.mark.parametrize("name", list(SPECS))
@pytest.mark.parametrize("n", [1, 1000, 100_003])
def test_sort_multi(tj, name, n):
    rng = np.random.default_rng(n + len(name))
    cols = _cols(rng, n, SPECS[name])
    if name.startswith("wide") and n > 10:
        # many equal tuples too: repeat a fifth of the rows
        k = n // 5
        for c in cols:
            c[-k:] = c[:k]
    rids = rng.permutation(n).astype(np.int32)
    outs, rout, st = tj.sort_multi([dev(c) for c in cols], dev(rids), stats=True)
    ec, er = multi.sort(cols, rids)
    assert np.array_equal(rout.cpu().numpy(), er)
    for o, e in zip(outs, ec):
        assert np.array_equal(o.cpu().numpy(), e)


def _join_inputs(rng, n_r, n_s, spec, dup=0.6):
    rc = _cols(rng, n_r, spec)
    sc = _cols(rng, n_s, spec)
    # a share of S tuples copied from R rows so that wide keys match
    m = int(n_s * dup)
    idx = rng.integers(0, n_r, m)
    for a, b in zip(rc, sc):
        b[:m] = a[idx]
    perm = rng.permutation(n_s)
    sc = [b[perm] for b in sc]
    return rc, sc


@pytest.mark.parametrize("name", ["packed32", "packed64", "wide2", "wide3", "constant"])
def test_join_multi(tj, name):
    rng = np.random.default_rng(len(name))
    rc, sc = _join_inputs(rng, 3000, 5000, SPECS[name])
    rr = rng.permutation(3000).astype(np.int32)
    sr = rng.permutation(5000).astype(np.int32)
    er, es, cnt = multi.join_pairs(rc, rr, sc, sr)
    assert tj.join_count_multi([dev(c) for c in rc], [dev(c) for c in sc]) == cnt
    pr, ps = tj.join_multi([dev(c) for c in rc], dev(rr), [dev(c) for c in sc], dev(sr), capacity=cnt)
    assert np.array_equal(pr.cpu().numpy(), er) and np.array_equal(ps.cpu().numpy(), es)


def test_join_multi_larger_dense_rank(tj):
    rng = np.random.default_rng(77)
    rc, sc = _join_inputs(rng, 60_000, 90_000, SPECS["wide2"], dup=0.5)
    rr = np.arange(60_000, dtype=np.int32)
    sr = np.arange(90_000, dtype=np.int32)
    er, es, cnt = multi.join_pairs(rc, rr, sc, sr)
    pr, ps, st = tj.join_multi([dev(c) for c in rc], dev(rr), [dev(c) for c in sc], dev(sr), capacity=cnt,
                               stats=True)
    assert np.array_equal(pr.cpu().numpy(), er) and np.array_equal(ps.cpu().numpy(), es)


def test_sort_multi_large(tj):
    n = 1 << 22
    rng = np.random.default_rng(5)
    cols = _cols(rng, n, [(0, 1000, np.int32), (I64.min, I64.max, np.int64), (-3, 3, np.int32)])
    rids = np.arange(n, dtype=np.int32)
    outs, rout = tj.sort_multi([dev(c) for c in cols], dev(rids))
    ec, er = multi.sort(cols, rids)
    assert np.array_equal(rout.cpu().numpy(), er)

"""Tests of the seeded input generators (no GPU needed)."""
import numpy as np

import tjgen


def test_splitmix64_reference_values():
    # SplitMix64 seeded with 0: the first outputs of the published generator
    assert tjgen.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert tjgen.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert tjgen.splitmix64(0, 2) == 0x06C45D188009454F


def test_bijection_exhaustive_20_bits():
    # a permutation of [0, 2^20) needs no cycle walking: it is the 20-bit
    # bijection itself, so this checks that bijection exhaustively
    n = 1 << 20
    out = tjgen.perm_i32(n, 99)
    assert np.array_equal(np.sort(out), np.arange(n, dtype=np.int32))
    assert all(tjgen.bij(20, 99, x) == out[x] for x in (0, 1, 12345, n - 1))


def test_permutation_non_power_of_two():
    for n in (1, 2, 3, 5, 1000, 12345):
        p = tjgen.perm_i32(n, 7)
        assert np.array_equal(np.sort(p), np.arange(n, dtype=np.int32))


def test_determinism():
    a = tjgen.paper_shaped(0.99, n=50_000)
    b = tjgen.paper_shaped(0.99, n=50_000)
    for k in a:
        assert np.array_equal(a[k], b[k])


def test_fk_structure():
    w = tjgen.paper_shaped(0.0, n=200_000)
    rk, sk = w["r_keys"], w["s_keys"]
    assert np.unique(rk).size == rk.size                      # unique R keys
    assert rk.min() >= 0 and rk.max() < (1 << 40)
    matched = np.isin(sk, rk)
    assert matched.sum() == int(0.8 * sk.size)                # exactly 80% match
    assert np.unique(sk[~matched]).size == (~matched).sum()   # fresh keys are distinct


def test_multiplicity_structure():
    w = tjgen.hbm_scale(0.99, n_r=1 << 14, n_s=1 << 16, hot=1 << 8, mult=4)
    u, c = np.unique(w["r_keys"], return_counts=True)
    assert (c == 4).sum() == 1 << 8 and (c == 1).sum() == (1 << 14) - 4 * (1 << 8)


def test_zipf_head_frequencies():
    d, m, theta = 1000, 400_000, 0.99
    z = tjgen.zipf_ranks(m, theta, d, 5)
    assert z.max() < d
    freq = np.bincount(z.astype(np.int64), minlength=d) / m
    p = np.arange(1, d + 1, dtype=np.float64) ** -theta
    p /= p.sum()
    # head ranks within 5 standard errors
    for r in range(10):
        se = np.sqrt(p[r] * (1 - p[r]) / m)
        assert abs(freq[r] - p[r]) < 5 * se
    u = tjgen.zipf_ranks(m, 0.0, d, 5)
    assert abs(np.bincount(u.astype(np.int64), minlength=d).std() / (m / d)) < 0.1


def test_learned_workloads_deterministic_and_shaped():
    n = 1 << 16
    for d in tjgen.LEARNED_DISTS:
        a, b = tjgen.learned(d, n), tjgen.learned(d, n)
        for c in ("r_keys", "s_keys", "r_rids", "s_rids"):
            assert np.array_equal(a[c], b[c]), (d, c)
        assert a["r_keys"].dtype == np.int64 and len(a["s_keys"]) == n
        assert (a["r_keys"] >= 0).all() and (a["s_keys"] >= 0).all()
        # 80% of S rows copy an R key (fresh draws may add a few more matches)
        frac = np.isin(a["s_keys"], a["r_keys"]).mean()
        assert 0.79 <= frac <= 0.85, (d, frac)


def test_lognormal_moments():
    k = tjgen.lognormal_i64(1 << 18, tjgen.stream(5))
    lk = np.log(k.astype(np.float64) + 0.5)
    assert abs(lk.mean() - 30.0) < 0.02 and abs(lk.std() - 2.0) < 0.02


def test_mixture_rows_stay_in_their_intervals():
    k, comp = tjgen.mixture_i64(1 << 17, tjgen.stream(6))
    lo, width, w = comp[:, 0], comp[:, 1], comp[:, 2]
    assert np.all((width >= 2.0 ** 20) & (width <= 2.0 ** 50)) and np.all(lo < 2.0 ** 62)
    inside = np.zeros(len(k), dtype=bool)
    hits = []
    for c in range(len(lo)):
        m = (k >= lo[c]) & (k <= lo[c] + width[c])
        inside |= m
        hits.append(m.mean())
    assert inside.all()
    # row shares follow the Dirichlet weights (components may overlap: lower bound only)
    assert all(h >= wc / w.sum() - 0.01 for h, wc in zip(hits, w))


def test_seqgap_is_a_shuffled_increasing_sequence():
    n = 1 << 16
    k = tjgen.seqgap_i64(n, tjgen.stream(7))
    s = np.sort(k)
    g = np.diff(s)
    assert g.min() >= 1 and abs(g.mean() - 8.0) < 0.1  # 1 + Geometric(1/8): mean 8
    assert not np.array_equal(k, s)  # shuffled

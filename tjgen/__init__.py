"""Seeded synthetic inputs for the equi-join and sort workloads.

The arrays built here feed both the CPU oracle and the GPU path; this module
holds none of the join or sort arithmetic.  The generators are counter based
(SplitMix64), so output depends only on the seed, never on thread count.

Workload recipes (the relation shapes, key domains and skew follow the paper's
evaluation setting of Sec. V, N = 1,000,000 rows and a work_mem budget, scaled
as stated for each recipe):

* ``small_uniform``  R, S of 100,000 rows, int32 keys uniform in [0, 2^20),
  row id = position.
* ``paper_shaped``   |R| = |S| = 1,000,000, int64 keys. R keys are unique and
  spread over [0, 2^40) by a bijection; S is foreign-key style: 80% of its rows
  take an R key chosen by Zipf(theta) over R's distinct keys (theta = 0 means
  uniform), 20% take fresh keys that no R row holds.  |R join S| = 800,000.
* ``hbm_scale``      |R| = 2^27, |S| = 2^29, same construction. The skewed
  variant gives the 2^20 hottest keys multiplicity 4 in R, so the join size
  is at most 4|S|; the generator returns the exact size.
* ``sort_uniform64`` n int64 keys uniform over the full 64-bit range.
* ``learned``        |R| = |S| = n (2^28 at full size), int64 keys from one of
  three non-uniform distributions: lognormal(mu = 30, sigma = 2) floored;
  a mixture of 8 uniform intervals placed uniformly in [0, 2^62) with widths
  2^20 ... 2^50 (log-uniform) and Dirichlet(1) weights; sequential keys with
  1 + Geometric(1/8) gaps, shuffled. S: 80% of its rows copy the key of a
  uniformly chosen R row, 20% are fresh draws of the same distribution (a
  fresh draw may coincide with an R key; the join size is not known in closed
  form). Row ids are positions.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

BASE_SEED = 260221237
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tjgen.c")
_LIB = os.path.join(_HERE, "libtjgen.so")
_lib = None

u64 = ctypes.c_uint64
_P = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile libtjgen.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.tjgen_splitmix64.restype = u64
        lib.tjgen_splitmix64.argtypes = [u64, u64]
        lib.tjgen_stream.restype = u64
        lib.tjgen_stream.argtypes = [u64, u64]
        lib.tjgen_bij.restype = u64
        lib.tjgen_bij.argtypes = [ctypes.c_uint, u64, u64]
        lib.tjgen_perm_at.restype = u64
        lib.tjgen_perm_at.argtypes = [u64, u64, u64]
        lib.tjgen_zipf_ranks.restype = None
        lib.tjgen_zipf_ranks.argtypes = [_P, u64, ctypes.c_double, u64, u64]
        lib.tjgen_uniform_i32.argtypes = [_P, u64, u64, ctypes.c_uint]
        lib.tjgen_uniform_i64.argtypes = [_P, u64, u64, ctypes.c_uint]
        lib.tjgen_perm_i32.argtypes = [_P, u64, u64]
        lib.tjgen_iota_i32.argtypes = [_P, u64]
        lib.tjgen_r_keys40.argtypes = [_P, u64, u64, u64, u64, u64]
        lib.tjgen_s_keys40.restype = u64
        lib.tjgen_s_keys40.argtypes = [_P, u64, u64, u64, u64, u64, ctypes.c_double, u64, u64, u64]
        lib.tjgen_lognormal_i64.argtypes = [_P, u64, u64, ctypes.c_double, ctypes.c_double]
        lib.tjgen_mixture_i64.argtypes = [_P, u64, u64, ctypes.c_uint, ctypes.c_double, ctypes.c_double, _P]
        lib.tjgen_seqgap_i64.argtypes = [_P, u64, u64, ctypes.c_double]
        lib.tjgen_fk_from.argtypes = [_P, u64, u64, _P, u64, _P, u64]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def stream(tag: int, seed: int = BASE_SEED) -> int:
    return int(_load().tjgen_stream(seed, tag))


def splitmix64(seed: int, i: int) -> int:
    return int(_load().tjgen_splitmix64(seed, i))


def bij(k: int, seed: int, x: int) -> int:
    return int(_load().tjgen_bij(k, seed, x))


def perm_at(n: int, seed: int, i: int) -> int:
    return int(_load().tjgen_perm_at(n, seed, i))


def zipf_ranks(m: int, theta: float, d: int, seed: int) -> np.ndarray:
    out = np.empty(m, dtype=np.uint64)
    _load().tjgen_zipf_ranks(_ptr(out), m, theta, d, seed)
    return out


def uniform_i32(n: int, seed: int, bits: int = 32) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().tjgen_uniform_i32(_ptr(out), n, seed, bits)
    return out


def uniform_i64(n: int, seed: int, bits: int = 64) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _load().tjgen_uniform_i64(_ptr(out), n, seed, bits)
    return out


def perm_i32(n: int, seed: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().tjgen_perm_i32(_ptr(out), n, seed)
    return out


def iota_i32(n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().tjgen_iota_i32(_ptr(out), n)
    return out


def r_keys40(n_r: int, hot: int, mult: int, key_seed: int, perm_seed: int) -> np.ndarray:
    out = np.empty(n_r, dtype=np.int64)
    _load().tjgen_r_keys40(_ptr(out), n_r, hot, mult, key_seed, perm_seed)
    return out


def s_keys40(n_s: int, n_matched: int, d_keys: int, hot: int, mult: int, theta: float,
             key_seed: int, perm_seed: int, zipf_seed: int):
    out = np.empty(n_s, dtype=np.int64)
    total = _load().tjgen_s_keys40(_ptr(out), n_s, n_matched, d_keys, hot, mult, theta,
                                   key_seed, perm_seed, zipf_seed)
    return out, int(total)


class Workload(dict):
    """A dict of host arrays plus metadata (name, expected join size when known)."""


def _fk_pair(tag: int, n_r: int, n_s: int, theta: float, hot: int = 0, mult: int = 1,
             matched_frac: float = 0.8, rid_perm: bool = False, seed: int = BASE_SEED) -> Workload:
    key_seed = stream(tag * 16 + 1, seed)
    d_keys = n_r - hot * (mult - 1)
    rk = r_keys40(n_r, hot, mult, key_seed, stream(tag * 16 + 2, seed))
    n_matched = int(n_s * matched_frac)  # floor
    sk, count = s_keys40(n_s, n_matched, d_keys, hot, mult, theta, key_seed,
                         stream(tag * 16 + 3, seed), stream(tag * 16 + 4, seed))
    if rid_perm:
        rr = perm_i32(n_r, stream(tag * 16 + 5, seed))
        sr = perm_i32(n_s, stream(tag * 16 + 6, seed))
    else:
        rr = iota_i32(n_r)
        sr = iota_i32(n_s)
    w = Workload(r_keys=rk, r_rids=rr, s_keys=sk, s_rids=sr)
    w.expected_count = count
    w.distinct_r = d_keys
    return w


def small_uniform(seed: int = BASE_SEED, n: int = 100_000, bits: int = 20,
                  rid_perm: bool = False) -> Workload:
    """R and S of n rows, int32 keys uniform in [0, 2^bits), row id = position."""
    rk = uniform_i32(n, stream(11, seed), bits)
    sk = uniform_i32(n, stream(12, seed), bits)
    if rid_perm:
        rr, sr = perm_i32(n, stream(13, seed)), perm_i32(n, stream(14, seed))
    else:
        rr, sr = iota_i32(n), iota_i32(n)
    w = Workload(r_keys=rk, r_rids=rr, s_keys=sk, s_rids=sr)
    w.expected_count = None
    return w


def paper_shaped(theta: float = 0.0, seed: int = BASE_SEED, n: int = 1_000_000,
                 rid_perm: bool = False) -> Workload:
    """|R| = |S| = n, unique 40-bit R keys, 80% FK matches with Zipf(theta)."""
    return _fk_pair(20 + int(round(theta * 100)), n, n, theta, rid_perm=rid_perm, seed=seed)


def hbm_scale(theta: float = 0.0, seed: int = BASE_SEED, n_r: int = 1 << 27,
              n_s: int = 1 << 29, hot: int | None = None, mult: int = 4) -> Workload:
    """|R| = 2^27, |S| = 2^29. theta > 0 adds multiplicity `mult` to the 2^20 hottest keys."""
    if hot is None:
        hot = (1 << 20) if theta > 0 else 0
    return _fk_pair(40 + int(round(theta * 100)), n_r, n_s, theta, hot=hot, mult=mult, seed=seed)


def crossover(lg: int, seed: int = BASE_SEED) -> Workload:
    """|R| = |S| = 2^lg, the paper-shaped structure (unique 40-bit R keys, 80%
    uniform FK matches): the inputs of the path-selection size sweep."""
    n = 1 << lg
    return _fk_pair(300 + lg, n, n, 0.0, seed=seed)


def sort_uniform64(n: int = 1 << 29, seed: int = BASE_SEED, bits: int = 64) -> Workload:
    """n int64 keys uniform over [0, 2^bits) (bits = 64: the whole signed range)."""
    w = Workload(keys=uniform_i64(n, stream(60 + bits, seed), bits), rids=iota_i32(n))
    return w


def lognormal_i64(n: int, seed: int, mu: float = 30.0, sigma: float = 2.0) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _load().tjgen_lognormal_i64(_ptr(out), n, seed, mu, sigma)
    return out


def mixture_i64(n: int, seed: int, ncomp: int = 8, wlo: float = 20.0, whi: float = 50.0):
    """Keys and the (lo, width, weight) rows of the components."""
    out = np.empty(n, dtype=np.int64)
    comp = np.zeros((ncomp, 3), dtype=np.float64)
    _load().tjgen_mixture_i64(_ptr(out), n, seed, ncomp, wlo, whi, _ptr(comp))
    return out, comp


def seqgap_i64(n: int, seed: int, p: float = 0.125) -> np.ndarray:
    out = np.empty(n, dtype=np.int64)
    _load().tjgen_seqgap_i64(_ptr(out), n, seed, p)
    return out


LEARNED_DISTS = ("lognormal", "mixture", "seqgap")


def _learned_keys(dist: str, n: int, seed: int) -> np.ndarray:
    if dist == "lognormal":
        return lognormal_i64(n, seed)
    if dist == "mixture":
        return mixture_i64(n, seed)[0]
    if dist == "seqgap":
        return seqgap_i64(n, seed)
    raise ValueError("unknown distribution %r" % dist)


def learned(dist: str, n: int = 1 << 28, seed: int = BASE_SEED, matched_frac: float = 0.8) -> Workload:
    """R and S of n rows each with keys of distribution `dist` (LEARNED_DISTS)."""
    tag = 80 + LEARNED_DISTS.index(dist)
    rk = _learned_keys(dist, n, stream(tag * 16 + 1, seed))
    n_matched = int(n * matched_frac)
    if dist == "mixture":
        # fresh S draws come from the same components (same component seed), new row counters
        fresh = _learned_keys_offset(dist, n - n_matched, stream(tag * 16 + 1, seed), n)
    elif dist == "seqgap":
        # fresh keys continue the same process past R's largest key
        fresh = seqgap_i64(n - n_matched, stream(tag * 16 + 2, seed)) + (int(rk.max()) if n else 0)
    else:
        fresh = _learned_keys(dist, n - n_matched, stream(tag * 16 + 2, seed))
    sk = np.empty(n, dtype=np.int64)
    _load().tjgen_fk_from(_ptr(sk), n, n_matched, _ptr(rk), n, _ptr(fresh), stream(tag * 16 + 3, seed))
    w = Workload(r_keys=rk, r_rids=iota_i32(n), s_keys=sk, s_rids=iota_i32(n))
    w.expected_count = None
    w.dist = dist
    return w


def _learned_keys_offset(dist: str, n: int, seed: int, skip: int) -> np.ndarray:
    """Rows skip .. skip + n - 1 of the mixture stream `seed` (same components)."""
    allk = mixture_i64(skip + n, seed)[0]
    return np.ascontiguousarray(allk[skip:])

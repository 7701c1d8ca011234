"""CPU oracle for the tensor-path sort and equi-join (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package. It shares no code with the GPU library and imports nothing from
it. The definitions it computes (see tj_oracle.cpp):

* sort:   stable ascending order by signed key, row ids carried (Sec. IV.B);
* count:  |R join S| = sum_k cnt_R(k) * cnt_S(k) (Sec. IV.A);
* pairs:  all (rid_R, rid_S) with equal keys, ordered by key, then R input
          position, then S input position (Sec. IV.A, late materialisation of
          Sec. III.A).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tj_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
_u64 = ctypes.c_uint64
_P = ctypes.c_void_p


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (single-threaded, -O3)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def build_native(out_dir: str) -> str:
    """Compile the same source with -O3 -march=native into out_dir, for timing
    on the machine that runs it (the benchmark's CPU leg)."""
    path = os.path.join(out_dir, "liboracle_native.so")
    subprocess.check_call(["g++", "-O3", "-march=native", "-std=c++17", "-shared", "-fPIC", "-o", path, _SRC])
    return path


def _bind(lib):
    for t in ("i32", "i64"):
        getattr(lib, "tjo_sort_" + t).argtypes = [_P, _P, _u64, _P, _P]
        f = getattr(lib, "tjo_join_count_" + t)
        f.argtypes, f.restype = [_P, _u64, _P, _u64], _u64
        f = getattr(lib, "tjo_join_pairs_" + t)
        f.argtypes, f.restype = [_P, _P, _u64, _P, _P, _u64, _P, _P, _u64], _u64
        f = getattr(lib, "tjo_pairs_for_key_" + t)
        kt = ctypes.c_int32 if t == "i32" else ctypes.c_int64
        f.argtypes, f.restype = [kt, _P, _P, _u64, _P, _P, _u64, _P, _P, _u64], _u64
    return lib


def _sfx(keys: np.ndarray) -> str:
    if keys.dtype == np.int32:
        return "i32"
    if keys.dtype == np.int64:
        return "i64"
    raise TypeError("keys must be int32 or int64, got %s" % keys.dtype)


def _c(a: np.ndarray, dtype) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, a.dtype))
    return a


class Oracle:
    """The oracle functions bound to one compiled library (the default one, or
    a deliberately mutated copy built by the tests to show the pins bite)."""

    def __init__(self, path: str):
        self.lib = _bind(ctypes.CDLL(path))

    def sort(self, keys: np.ndarray, rids: np.ndarray):
        """Stable ascending sort by signed key; returns (keys_out, rids_out)."""
        sfx = _sfx(keys)
        keys = _c(keys, keys.dtype)
        rids = _c(rids, np.int32)
        assert keys.shape == rids.shape
        ko = np.empty_like(keys)
        ro = np.empty_like(rids)
        getattr(self.lib, "tjo_sort_" + sfx)(keys.ctypes.data, rids.ctypes.data, keys.size,
                                             ko.ctypes.data, ro.ctypes.data)
        return ko, ro

    def join_count(self, r_keys: np.ndarray, s_keys: np.ndarray) -> int:
        """|R join S| on equal keys."""
        sfx = _sfx(r_keys)
        r_keys = _c(r_keys, r_keys.dtype)
        s_keys = _c(s_keys, r_keys.dtype)
        return int(getattr(self.lib, "tjo_join_count_" + sfx)(r_keys.ctypes.data, r_keys.size,
                                                               s_keys.ctypes.data, s_keys.size))

    def join_pairs(self, r_keys, r_rids, s_keys, s_rids, capacity: int | None = None):
        """All matching (rid_R, rid_S) in canonical order; returns (out_r, out_s, count)."""
        sfx = _sfx(r_keys)
        r_keys = _c(r_keys, r_keys.dtype)
        s_keys = _c(s_keys, r_keys.dtype)
        r_rids = _c(r_rids, np.int32)
        s_rids = _c(s_rids, np.int32)
        f = getattr(self.lib, "tjo_join_pairs_" + sfx)
        if capacity is None:
            capacity = self.join_count(r_keys, s_keys)
        out_r = np.empty(max(capacity, 1), dtype=np.int32)
        out_s = np.empty(max(capacity, 1), dtype=np.int32)
        cnt = int(f(r_keys.ctypes.data, r_rids.ctypes.data, r_keys.size, s_keys.ctypes.data,
                    s_rids.ctypes.data, s_keys.size, out_r.ctypes.data, out_s.ctypes.data,
                    capacity))
        m = min(cnt, capacity)
        return out_r[:m], out_s[:m], cnt

    def pairs_for_key(self, key: int, r_keys, r_rids, s_keys, s_rids):
        """The pairs of one key in canonical order, by linear scans (sampled checks)."""
        sfx = _sfx(r_keys)
        f = getattr(self.lib, "tjo_pairs_for_key_" + sfx)
        r_keys = _c(r_keys, r_keys.dtype)
        s_keys = _c(s_keys, r_keys.dtype)
        r_rids = _c(r_rids, np.int32)
        s_rids = _c(s_rids, np.int32)
        cnt = int(f(key, r_keys.ctypes.data, r_rids.ctypes.data, r_keys.size,
                    s_keys.ctypes.data, s_rids.ctypes.data, s_keys.size, None, None, 0))
        out_r = np.empty(max(cnt, 1), dtype=np.int32)
        out_s = np.empty(max(cnt, 1), dtype=np.int32)
        f(key, r_keys.ctypes.data, r_rids.ctypes.data, r_keys.size, s_keys.ctypes.data,
          s_rids.ctypes.data, s_keys.size, out_r.ctypes.data, out_s.ctypes.data, cnt)
        return out_r[:cnt], out_s[:cnt]


def _default() -> Oracle:
    global _lib
    if _lib is None:
        _lib = Oracle(build())
    return _lib


def sort(keys, rids):
    return _default().sort(keys, rids)


def join_count(r_keys, s_keys) -> int:
    return _default().join_count(r_keys, s_keys)


def join_pairs(r_keys, r_rids, s_keys, s_rids, capacity=None):
    return _default().join_pairs(r_keys, r_rids, s_keys, s_rids, capacity)


def pairs_for_key(key, r_keys, r_rids, s_keys, s_rids):
    return _default().pairs_for_key(key, r_keys, r_rids, s_keys, s_rids)

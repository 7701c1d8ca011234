"""ctypes binding of libtj.so (include/tj.h): argument marshalling only.

Device memory and streams come from PyTorch; every step of the sort and join
runs in the library's HIP kernels. The functions take and return torch tensors
on a ROCm device. There is no fallback: if the library is not built, or no GPU
is visible, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libtj.so")

TJ_KEY_I32, TJ_KEY_I64 = 4, 8
TJ_OP_SORT, TJ_OP_JOIN_COUNT, TJ_OP_JOIN_MATERIALIZE = 0, 1, 2
TJ_STATIC_SCRATCH_BYTES = 256 << 20  # the device scratch of tj_sort_static
TJ_OK, TJ_E_ARG, TJ_E_WORKSPACE, TJ_E_CAPACITY = 0, -1, -2, -3
TJ_E_TOO_LARGE, TJ_E_ALIAS, TJ_E_HIP, TJ_E_INTERNAL = -4, -5, -6, -7

_u64 = ctypes.c_uint64
_P = ctypes.c_void_p
_lib = None


class TjError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, strerror(status) if _lib else "?", status))


class Stats(ctypes.Structure):
    _fields_ = [("bytes_read", ctypes.c_uint64), ("bytes_written", ctypes.c_uint64),
                ("workspace_used", ctypes.c_uint64), ("passes", ctypes.c_uint32),
                ("leaves", ctypes.c_uint32), ("single_key", ctypes.c_uint32),
                ("key_ranges", ctypes.c_uint32), ("learned", ctypes.c_uint32),
                ("learned_overflow", ctypes.c_uint32), ("windows", ctypes.c_uint32),
                ("pivots", ctypes.c_uint32), ("sample_rows", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


RMI_SEGMENTS, RMI_LEAVES = 256, 1024
TJ_PART_RADIX, TJ_PART_LEARNED, TJ_PART_AUTO = 0, 1, 2
_PARTITIONERS = {"radix": TJ_PART_RADIX, "learned": TJ_PART_LEARNED, "auto": TJ_PART_AUTO}


class RmiModel(ctypes.Structure):
    """tj_rmi_t: the learned bucket function (see include/tj.h)."""
    _fields_ = [("knot", ctypes.c_uint64 * (RMI_SEGMENTS + 1)), ("knot_inv", ctypes.c_float * RMI_SEGMENTS),
                ("leaf_base", ctypes.c_uint64 * RMI_LEAVES), ("leaf_a", ctypes.c_float * RMI_LEAVES),
                ("leaf_b", ctypes.c_float * RMI_LEAVES), ("leaf_lo", ctypes.c_uint16 * RMI_LEAVES),
                ("leaf_hi", ctypes.c_uint16 * RMI_LEAVES), ("buckets", ctypes.c_uint32),
                ("sample_rows", ctypes.c_uint32)]

    ARRAYS = ("knot", "knot_inv", "leaf_base", "leaf_a", "leaf_b", "leaf_lo", "leaf_hi")

    def to_numpy(self) -> dict:
        import numpy as np
        out = {f: np.ctypeslib.as_array(getattr(self, f)).copy() for f in self.ARRAYS}
        out["buckets"] = int(self.buckets)
        out["sample_rows"] = int(self.sample_rows)
        return out

    @classmethod
    def from_fields(cls, obj) -> "RmiModel":
        """From any object (or dict) with the model's field names as arrays / ints."""
        import numpy as np
        get = (lambda k: obj[k]) if isinstance(obj, dict) else (lambda k: getattr(obj, k))
        m = cls()
        for f in cls.ARRAYS:
            dst = np.ctypeslib.as_array(getattr(m, f))
            dst[:] = np.asarray(get(f), dtype=dst.dtype)
        m.buckets = int(get("buckets"))
        m.sample_rows = int(get("sample_rows"))
        return m


class Options(ctypes.Structure):
    _fields_ = [("partitioner", ctypes.c_uint32), ("sample_permille", ctypes.c_uint32),
                ("learned_min_rows", ctypes.c_uint64)]


def _options(partitioner: str, sample_permille: int, learned_min_rows: int):
    if partitioner not in _PARTITIONERS:
        raise ValueError("partitioner must be one of %s" % sorted(_PARTITIONERS))
    return Options(_PARTITIONERS[partitioner], sample_permille, learned_min_rows)


EXPORTS = {
    "tj_workspace_query": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _u64, _u64,
                                          ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "tj_sort": (ctypes.c_int, [ctypes.c_int, _P, _P, _u64, _P, _P, _P, _u64, _P, _P]),
    "tj_join_count": (ctypes.c_int, [ctypes.c_int, _P, _u64, _P, _u64, ctypes.POINTER(_u64),
                                     _P, _u64, _P, _P]),
    "tj_join_materialize": (ctypes.c_int, [ctypes.c_int, _P, _P, _u64, _P, _P, _u64, _P, _P, _u64,
                                           ctypes.POINTER(_u64), _P, _u64, _P, _P]),
    "tj_sort_ex": (ctypes.c_int, [ctypes.c_int, _P, _P, _u64, _P, _P, _P, _u64, _P, _P, _P]),
    "tj_sort_static": (ctypes.c_int, [ctypes.c_int, _P, _P, _u64, _P, _P, _P, _P]),
    "tj_join_count_ex": (ctypes.c_int, [ctypes.c_int, _P, _u64, _P, _u64, ctypes.POINTER(_u64),
                                        _P, _u64, _P, _P, _P]),
    "tj_join_materialize_ex": (ctypes.c_int, [ctypes.c_int, _P, _P, _u64, _P, _P, _u64, _P, _P, _u64,
                                              ctypes.POINTER(_u64), _P, _u64, _P, _P, _P]),
    "tj_rmi_workspace_query": (ctypes.c_int, [ctypes.c_int, _u64, _u64, ctypes.c_uint32,
                                              ctypes.POINTER(_u64)]),
    "tj_rmi_train": (ctypes.c_int, [ctypes.c_int, _P, _u64, _P, _u64, ctypes.c_uint32, _P, _P, _u64, _P]),
    "tj_rmi_buckets": (ctypes.c_int, [ctypes.c_int, _P, _u64, _P, _P, _P, _u64, _P]),
    "tj_multi_workspace_query": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _u64, _u64, ctypes.POINTER(_u64)]),
    "tj_sort_multi": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _u64, _P, _P, _P, _u64, _P, _P]),
    "tj_join_count_multi": (ctypes.c_int, [ctypes.c_int, _P, _P, _u64, _P, _u64, ctypes.POINTER(_u64), _P, _u64,
                                           _P, _P]),
    "tj_join_materialize_multi": (ctypes.c_int, [ctypes.c_int, _P, _P, _P, _u64, _P, _P, _u64, _P, _P, _u64,
                                                 ctypes.POINTER(_u64), _P, _u64, _P, _P]),
    "tj_server_create": (ctypes.c_int, [_P, _u64, ctypes.c_int, ctypes.POINTER(_P)]),
    "tj_server_submit": (ctypes.c_int, [_P, _P, ctypes.POINTER(_u64)]),
    "tj_server_wait": (ctypes.c_int, [_P, _u64, _P]),
    "tj_server_memory": (ctypes.c_int, [_P, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "tj_server_configure": (ctypes.c_int, [_P, _u64, ctypes.c_uint32]),
    "tj_server_destroy": (ctypes.c_int, [_P]),
    "tj_select_workspace_query": (ctypes.c_int, [_u64, _u64, ctypes.POINTER(_u64)]),
    "tj_select_path": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _P, _u64, _P, _u64, _P, _P, _P, _P, _u64, _P]),
    "tj_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "tj_version": (ctypes.c_int, []),
    "tj_timing": (ctypes.c_int, [ctypes.c_int]),
    "tj_timing_read": (ctypes.c_int, [_P, ctypes.c_int]),
    "tj_debug_wave_scan": (ctypes.c_int, [_P, _P, _u64, _P]),
    "tj_debug_set_flags": (ctypes.c_int, [ctypes.c_uint32]),
    "tj_debug_stream_copy": (ctypes.c_int, [_P, _P, _u64, _P]),
    "tj_debug_partition_pass": (ctypes.c_int, [_P, _P, _u64, _u64, ctypes.c_uint32, ctypes.c_uint32,
                                               ctypes.c_uint32, _P, _P, _P, _P, _u64, _P]),
}


def load(path: str = LIB_PATH):
    """Loads libtj.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libtj.so is not built (%s); run paper_2602_21237_amd.build.build()" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in EXPORTS.items():
            f = getattr(lib, name)
            f.restype, f.argtypes = res, args
        _lib = lib
    return _lib


def strerror(status: int) -> str:
    return load().tj_strerror(status).decode()


def _check(status: int, where: str):
    if status != TJ_OK:
        raise TjError(status, where)


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_uint64),
                ("bytes", ctypes.c_uint64), ("ms", ctypes.c_double)]


def timing(enable: bool) -> None:
    """Turns per-kernel HIP-event timing on (clearing the counters) or off."""
    _check(load().tj_timing(1 if enable else 0), "tj_timing")


def timing_read() -> dict:
    """{family: {"launches", "bytes", "ms"}} accumulated since timing(True)."""
    arr = (KernelStat * 32)()
    n = load().tj_timing_read(ctypes.cast(arr, ctypes.c_void_p), 32)
    if n < 0:
        raise TjError(n, "tj_timing_read")
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "bytes": int(arr[i].bytes),
                                   "ms": float(arr[i].ms)} for i in range(n)}


def workspace_query(op: int, key_type: int, n_r: int, n_s: int = 0):
    """(min_bytes, full_bytes) for an operation of this shape (host only)."""
    mn, full = _u64(), _u64()
    _check(load().tj_workspace_query(op, key_type, n_r, n_s, ctypes.byref(mn), ctypes.byref(full)),
           "tj_workspace_query")
    return int(mn.value), int(full.value)


# --------------------------------------------------------------------------- torch side

def _torch():
    import torch
    return torch


def _key_type(t) -> int:
    torch = _torch()
    if t.dtype == torch.int32:
        return TJ_KEY_I32
    if t.dtype == torch.int64:
        return TJ_KEY_I64
    raise TypeError("keys must be int32 or int64 tensors, got %s" % t.dtype)


def _dev(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(op, kt, n_r, n_s, workspace, workspace_bytes, device):
    torch = _torch()
    if workspace is not None:
        _dev(workspace, "workspace")
        nbytes = workspace.numel() * workspace.element_size()
        if workspace_bytes is None:
            workspace_bytes = nbytes
        if workspace_bytes > nbytes:
            raise ValueError("workspace_bytes exceeds the workspace tensor")
        return workspace, workspace_bytes
    mn, full = workspace_query(op, kt, n_r, n_s)
    if workspace_bytes is None:
        workspace_bytes = full
    ws = torch.empty(max(workspace_bytes, 256), dtype=torch.uint8, device=device)
    return ws, workspace_bytes


def sort(keys, rids, keys_out=None, rids_out=None, workspace=None, workspace_bytes=None,
         stream=None, stats: bool = False, partitioner: str = "radix", sample_permille: int = 0,
         learned_min_rows: int = 0):
    """Stable ascending sort of (keys, rids) by signed key (tj_sort, or tj_sort_ex
    with partitioner="learned")."""
    torch = _torch()
    _dev(keys, "keys")
    _dev(rids, "rids")
    if rids.dtype != torch.int32 or rids.shape != keys.shape:
        raise TypeError("rids must be int32 with the shape of keys")
    kt = _key_type(keys)
    n = keys.numel()
    if keys_out is None:
        keys_out = torch.empty_like(keys)
    if rids_out is None:
        rids_out = torch.empty_like(rids)
    ws, wsb = _workspace(TJ_OP_SORT, kt, n, 0, workspace, workspace_bytes, keys.device)
    st = Stats()
    if partitioner == "radix" and not sample_permille and not learned_min_rows:
        _check(load().tj_sort(kt, keys.data_ptr(), rids.data_ptr(), n, keys_out.data_ptr(),
                              rids_out.data_ptr(), ws.data_ptr(), wsb, _stream(stream), ctypes.byref(st)),
               "tj_sort")
    else:
        opt = _options(partitioner, sample_permille, learned_min_rows)
        _check(load().tj_sort_ex(kt, keys.data_ptr(), rids.data_ptr(), n, keys_out.data_ptr(),
                                 rids_out.data_ptr(), ws.data_ptr(), wsb, _stream(stream), ctypes.byref(opt),
                                 ctypes.byref(st)), "tj_sort_ex")
    return (keys_out, rids_out, st.as_dict()) if stats else (keys_out, rids_out)


def sort_static(keys, rids, keys_out, rids_out, stream=None, stats: bool = False):
    """tj_sort_static: the sort of tj_sort on the library's own device scratch.
    Outputs are the caller's (allocated beforehand); the call allocates nothing."""
    torch = _torch()
    _dev(keys, "keys")
    _dev(rids, "rids")
    _dev(keys_out, "keys_out")
    _dev(rids_out, "rids_out")
    if rids.dtype != torch.int32 or rids.shape != keys.shape:
        raise TypeError("rids must be int32 with the shape of keys")
    if keys_out.dtype != keys.dtype or keys_out.shape != keys.shape or rids_out.dtype != torch.int32 \
            or rids_out.shape != keys.shape:
        raise TypeError("outputs must match the inputs' shapes and types")
    st = Stats()
    _check(load().tj_sort_static(_key_type(keys), keys.data_ptr(), rids.data_ptr(), keys.numel(),
                                 keys_out.data_ptr(), rids_out.data_ptr(), _stream(stream), ctypes.byref(st)),
           "tj_sort_static")
    return st.as_dict() if stats else None


def join_count(r_keys, s_keys, workspace=None, workspace_bytes=None, stream=None,
               stats: bool = False, partitioner: str = "radix", sample_permille: int = 0,
               learned_min_rows: int = 0):
    """|R join S| on equal keys (tj_join_count, or tj_join_count_ex with options)."""
    _dev(r_keys, "r_keys")
    _dev(s_keys, "s_keys")
    kt = _key_type(r_keys)
    if _key_type(s_keys) != kt:
        raise TypeError("r_keys and s_keys must have the same dtype")
    ws, wsb = _workspace(TJ_OP_JOIN_COUNT, kt, r_keys.numel(), s_keys.numel(), workspace,
                         workspace_bytes, r_keys.device)
    cnt = _u64()
    st = Stats()
    if partitioner == "radix" and not sample_permille and not learned_min_rows:
        _check(load().tj_join_count(kt, r_keys.data_ptr(), r_keys.numel(), s_keys.data_ptr(),
                                    s_keys.numel(), ctypes.byref(cnt), ws.data_ptr(), wsb,
                                    _stream(stream), ctypes.byref(st)), "tj_join_count")
    else:
        opt = _options(partitioner, sample_permille, learned_min_rows)
        _check(load().tj_join_count_ex(kt, r_keys.data_ptr(), r_keys.numel(), s_keys.data_ptr(),
                                       s_keys.numel(), ctypes.byref(cnt), ws.data_ptr(), wsb,
                                       _stream(stream), ctypes.byref(opt), ctypes.byref(st)), "tj_join_count_ex")
    return (int(cnt.value), st.as_dict()) if stats else int(cnt.value)


def join(r_keys, r_rids, s_keys, s_rids, capacity: int | None = None, out_r=None, out_s=None,
         workspace=None, workspace_bytes=None, stream=None, stats: bool = False, partitioner: str = "radix",
         sample_permille: int = 0, learned_min_rows: int = 0):
    """All (rid_R, rid_S) pairs with equal keys in canonical order (tj_join_materialize).

    Returns (out_r[:count], out_s[:count]) (plus the stats dict). With
    capacity=None the count is taken first with tj_join_count."""
    torch = _torch()
    for t, nm in ((r_keys, "r_keys"), (r_rids, "r_rids"), (s_keys, "s_keys"), (s_rids, "s_rids")):
        _dev(t, nm)
    kt = _key_type(r_keys)
    if _key_type(s_keys) != kt or r_rids.dtype != torch.int32 or s_rids.dtype != torch.int32:
        raise TypeError("dtype mismatch")
    if capacity is None:
        capacity = out_r.numel() if out_r is not None else join_count(
            r_keys, s_keys, stream=stream, partitioner=partitioner, sample_permille=sample_permille,
            learned_min_rows=learned_min_rows)
    if out_r is None:
        out_r = torch.empty(max(capacity, 1), dtype=torch.int32, device=r_keys.device)
    if out_s is None:
        out_s = torch.empty(max(capacity, 1), dtype=torch.int32, device=r_keys.device)
    if out_r.numel() < capacity or out_s.numel() < capacity:
        raise ValueError("output tensors smaller than capacity")
    ws, wsb = _workspace(TJ_OP_JOIN_MATERIALIZE, kt, r_keys.numel(), s_keys.numel(), workspace,
                         workspace_bytes, r_keys.device)
    cnt = _u64()
    st = Stats()
    args = (kt, r_keys.data_ptr(), r_rids.data_ptr(), r_keys.numel(), s_keys.data_ptr(), s_rids.data_ptr(),
            s_keys.numel(), out_r.data_ptr(), out_s.data_ptr(), capacity, ctypes.byref(cnt), ws.data_ptr(), wsb,
            _stream(stream))
    if partitioner == "radix" and not sample_permille and not learned_min_rows:
        _check(load().tj_join_materialize(*args, ctypes.byref(st)), "tj_join_materialize")
    else:
        opt = _options(partitioner, sample_permille, learned_min_rows)
        _check(load().tj_join_materialize_ex(*args, ctypes.byref(opt), ctypes.byref(st)), "tj_join_materialize_ex")
    c = int(cnt.value)
    res = (out_r[:c], out_s[:c])
    return res + (st.as_dict(),) if stats else res


# --------------------------------------------------------------------------- composite keys

def _col_arrays(cols):
    cols = list(cols)
    for i, c in enumerate(cols):
        _dev(c, "key column %d" % i)
    types = (ctypes.c_int * len(cols))(*[_key_type(c) for c in cols])
    ptrs = (ctypes.c_void_p * len(cols))(*[c.data_ptr() for c in cols])
    return types, ptrs


def multi_workspace_query(op: int, cols, n_r: int, n_s: int = 0) -> int:
    types = (ctypes.c_int * len(cols))(*[_key_type(c) for c in cols])
    b = _u64()
    _check(load().tj_multi_workspace_query(op, len(cols), types, n_r, n_s, ctypes.byref(b)),
           "tj_multi_workspace_query")
    return int(b.value)


def sort_multi(cols, rids, workspace_bytes=None, stream=None, stats: bool = False):
    """Stable lexicographic sort of rows by key columns cols[0], cols[1], ...
    (tj_sort_multi). Returns (sorted columns, rids)."""
    torch = _torch()
    types, ptrs = _col_arrays(cols)
    _dev(rids, "rids")
    n = rids.numel()
    outs = [torch.empty_like(c) for c in cols]
    optrs = (ctypes.c_void_p * len(cols))(*[o.data_ptr() for o in outs])
    rout = torch.empty_like(rids)
    need = multi_workspace_query(TJ_OP_SORT, cols, n) if workspace_bytes is None else workspace_bytes
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=rids.device)
    st = Stats()
    _check(load().tj_sort_multi(len(cols), types, ptrs, rids.data_ptr(), n, optrs, rout.data_ptr(), ws.data_ptr(),
                                need, _stream(stream), ctypes.byref(st)), "tj_sort_multi")
    return (outs, rout, st.as_dict()) if stats else (outs, rout)


def join_count_multi(r_cols, s_cols, workspace_bytes=None, stream=None, stats: bool = False):
    """Equi-join size on all key columns (tj_join_count_multi)."""
    torch = _torch()
    rt, rp = _col_arrays(r_cols)
    _, sp = _col_arrays(s_cols)
    n_r, n_s = r_cols[0].numel(), s_cols[0].numel()
    need = multi_workspace_query(TJ_OP_JOIN_COUNT, r_cols, n_r, n_s) if workspace_bytes is None else workspace_bytes
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=r_cols[0].device)
    cnt = _u64()
    st = Stats()
    _check(load().tj_join_count_multi(len(r_cols), rt, rp, n_r, sp, n_s, ctypes.byref(cnt), ws.data_ptr(), need,
                                      _stream(stream), ctypes.byref(st)), "tj_join_count_multi")
    return (int(cnt.value), st.as_dict()) if stats else int(cnt.value)


def join_multi(r_cols, r_rids, s_cols, s_rids, capacity: int | None = None, workspace_bytes=None, stream=None,
               stats: bool = False):
    """All (rid_R, rid_S) pairs equal on every key column, canonical order
    (tj_join_materialize_multi)."""
    torch = _torch()
    rt, rp = _col_arrays(r_cols)
    _, sp = _col_arrays(s_cols)
    n_r, n_s = r_cols[0].numel(), s_cols[0].numel()
    if capacity is None:
        capacity = join_count_multi(r_cols, s_cols, stream=stream)
    out_r = torch.empty(max(capacity, 1), dtype=torch.int32, device=r_rids.device)
    out_s = torch.empty(max(capacity, 1), dtype=torch.int32, device=r_rids.device)
    need = (multi_workspace_query(TJ_OP_JOIN_MATERIALIZE, r_cols, n_r, n_s) if workspace_bytes is None
            else workspace_bytes)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=r_rids.device)
    cnt = _u64()
    st = Stats()
    _check(load().tj_join_materialize_multi(len(r_cols), rt, rp, r_rids.data_ptr(), n_r, sp, s_rids.data_ptr(), n_s,
                                            out_r.data_ptr(), out_s.data_ptr(), capacity, ctypes.byref(cnt),
                                            ws.data_ptr(), need, _stream(stream), ctypes.byref(st)),
           "tj_join_materialize_multi")
    c = int(cnt.value)
    res = (out_r[:c], out_s[:c])
    return res + (st.as_dict(),) if stats else res


def rmi_workspace_query(key_type: int, n_a: int, n_b: int = 0, permille: int = 0) -> int:
    b = _u64()
    _check(load().tj_rmi_workspace_query(key_type, n_a, n_b, permille, ctypes.byref(b)), "tj_rmi_workspace_query")
    return int(b.value)


def rmi_train(keys_a, keys_b=None, permille: int = 0, stream=None) -> RmiModel:
    """Fits the learned bucket function to samples of one or two key columns (tj_rmi_train)."""
    torch = _torch()
    _dev(keys_a, "keys_a")
    kt = _key_type(keys_a)
    nb = 0
    pb = None
    if keys_b is not None:
        _dev(keys_b, "keys_b")
        if _key_type(keys_b) != kt:
            raise TypeError("keys_a and keys_b must have the same dtype")
        nb, pb = keys_b.numel(), keys_b.data_ptr()
    need = rmi_workspace_query(kt, keys_a.numel(), nb, permille)
    ws = torch.empty(need, dtype=torch.uint8, device=keys_a.device)
    m = RmiModel()
    _check(load().tj_rmi_train(kt, keys_a.data_ptr(), keys_a.numel(), pb, nb, permille, ctypes.byref(m),
                               ws.data_ptr(), need, _stream(stream)), "tj_rmi_train")
    return m


def rmi_buckets(keys, model: RmiModel, stream=None):
    """Bucket of every key under a host-side model (tj_rmi_buckets); int32 tensor."""
    torch = _torch()
    _dev(keys, "keys")
    kt = _key_type(keys)
    out = torch.empty(max(keys.numel(), 1), dtype=torch.int16, device=keys.device)
    ws = torch.empty(ctypes.sizeof(RmiModel) + 256, dtype=torch.uint8, device=keys.device)
    _check(load().tj_rmi_buckets(kt, keys.data_ptr(), keys.numel(), ctypes.byref(model), out.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream(stream)), "tj_rmi_buckets")
    return out[:keys.numel()].to(torch.int32) & 0xFFFF


TJ_PATH_LINEAR, TJ_PATH_TENSOR = 0, 1
TJ_SEL_SCALE, TJ_SEL_OUTPUT = 1, 2
SELECT_REGISTERS = 16384
TJ_SELECT_DEFAULT_MIN_ROWS = 1 << 11
TJ_SELECT_DEFAULT_MIN_OUTPUT = 1 << 10


class SelectOptions(ctypes.Structure):
    _fields_ = [("min_rows", ctypes.c_uint64), ("min_output", ctypes.c_uint64)]


class Selection(ctypes.Structure):
    _fields_ = [("n_r", ctypes.c_uint64), ("n_s", ctypes.c_uint64), ("distinct_r", ctypes.c_double),
                ("distinct_s", ctypes.c_double), ("distinct_union", ctypes.c_double),
                ("distinct_common", ctypes.c_double), ("est_output", ctypes.c_double),
                ("path", ctypes.c_int32), ("reasons", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def select_workspace_query(n_r: int, n_s: int = 0) -> int:
    b = _u64()
    _check(load().tj_select_workspace_query(n_r, n_s, ctypes.byref(b)), "tj_select_workspace_query")
    return int(b.value)


def select_path(r_keys, s_keys=None, min_rows: int = 0, min_output: int = 0, registers=None, workspace=None,
                stream=None) -> dict:
    """Execution-time choice between the linear and the tensor path for a sort
    (s_keys None) or a join of the key columns (tj_select_path): the
    indicators and the decision as a dict. `registers`, when given, is a
    device uint8 tensor of 3 * 16384 bytes that receives the R, S and union
    HyperLogLog registers."""
    torch = _torch()
    _dev(r_keys, "r_keys")
    kt = _key_type(r_keys)
    op, n_s, ps = TJ_OP_SORT, 0, None
    if s_keys is not None:
        _dev(s_keys, "s_keys")
        if _key_type(s_keys) != kt:
            raise TypeError("r_keys and s_keys must have the same dtype")
        op, n_s, ps = TJ_OP_JOIN_COUNT, s_keys.numel(), s_keys.data_ptr()
    need = select_workspace_query(r_keys.numel(), n_s)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=r_keys.device)
    if registers is not None:
        _dev(registers, "registers")
        if registers.dtype != torch.uint8 or registers.numel() < 3 * SELECT_REGISTERS:
            raise ValueError("registers must be a uint8 tensor of at least 3 * 16384 elements")
    opt = SelectOptions(min_rows, min_output)
    out = Selection()
    _check(load().tj_select_path(op, kt, r_keys.data_ptr(), r_keys.numel(), ps, n_s, ctypes.byref(opt),
                                 ctypes.byref(out), registers.data_ptr() if registers is not None else None,
                                 workspace.data_ptr(), workspace.numel(), _stream(stream)), "tj_select_path")
    return out.as_dict()


def debug_wave_scan(x):
    """Inclusive prefix sum within each 64-lane wavefront (uint32 values in an int32 tensor)."""
    out = _torch().empty_like(x)
    _check(load().tj_debug_wave_scan(x.data_ptr(), out.data_ptr(), x.numel(), _stream(None)),
           "tj_debug_wave_scan")
    return out


TJ_DEBUG_FORCE_REORDER = 1
TJ_DEBUG_FAIL_HOST_ALLOC = 2


def debug_stream_copy(src, dst, stream=None) -> None:
    """Plain streaming copy of src into dst (device tensors of equal byte size,
    a multiple of 16 bytes), on `stream` (default: torch's current stream)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise ValueError("src and dst differ in size")
    _check(load().tj_debug_stream_copy(src.data_ptr(), dst.data_ptr(), nb, _stream(stream)),
           "tj_debug_stream_copy")


def debug_set_flags(flags: int) -> None:
    """Process-wide self-test flags for later calls (TJ_DEBUG_FORCE_REORDER,
    TJ_DEBUG_FAIL_HOST_ALLOC, or 0)."""
    _check(load().tj_debug_set_flags(flags), "tj_debug_set_flags")


def debug_partition_pass(keys, rids, base: int, shift: int, bits: int, workspace_bytes: int = 64 << 20,
                         force_reorder: bool = False):
    """One stable radix partition pass (int64 keys); returns (keys_out, rids_out, counts).
    force_reorder sends every tile through the scatter's re-ranking path."""
    torch = _torch()
    ko, ro = torch.empty_like(keys), torch.empty_like(rids)
    counts = torch.empty(1 << bits, dtype=torch.int32, device=keys.device)
    ws = torch.empty(workspace_bytes, dtype=torch.uint8, device=keys.device)
    _check(load().tj_debug_partition_pass(keys.data_ptr(), rids.data_ptr(), keys.numel(), base, shift,
                                          bits, TJ_DEBUG_FORCE_REORDER if force_reorder else 0,
                                          ko.data_ptr(), ro.data_ptr(), counts.data_ptr(),
                                          ws.data_ptr(), workspace_bytes, _stream(None)),
           "tj_debug_partition_pass")
    return ko, ro, counts


# --------------------------------------------------------------------------- serving loop

class Request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("key_type", ctypes.c_int), ("r_keys", _P), ("r_rids", _P),
                ("n_r", _u64), ("s_keys", _P), ("s_rids", _P), ("n_s", _u64), ("out0", _P), ("out1", _P),
                ("capacity", _u64), ("partitioner", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("op", ctypes.c_int), ("count", _u64),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("learned", ctypes.c_uint32), ("key_ranges", ctypes.c_uint32),
                ("fused", ctypes.c_uint32), ("windows", ctypes.c_uint32)]


class Server:
    """tj_server_*: requests run on `slots` concurrent streams, admitted against
    a device arena of `arena_bytes` that holds their workspaces. Inputs and
    outputs are device tensors the caller owns; the server keeps references to
    them until wait() returns."""

    def __init__(self, arena_bytes: int, slots: int = 4, device=None):
        torch = _torch()
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=device or "cuda")
        torch.cuda.synchronize()
        self._h = _P()
        _check(load().tj_server_create(self.arena.data_ptr(), arena_bytes, slots, ctypes.byref(self._h)),
               "tj_server_create")
        self._keep = {}

    def _submit(self, op, r_keys, r_rids, s_keys, s_rids, out0, out1, capacity, partitioner):
        kt = _key_type(r_keys)
        ptr = lambda t: t.data_ptr() if t is not None else None
        req = Request(op, kt, ptr(r_keys), ptr(r_rids), r_keys.numel(), ptr(s_keys), ptr(s_rids),
                      s_keys.numel() if s_keys is not None else 0, ptr(out0), ptr(out1), capacity,
                      _PARTITIONERS[partitioner], 0)
        t = _u64()
        _check(load().tj_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "tj_server_submit")
        self._keep[t.value] = (op, (r_keys, r_rids, s_keys, s_rids), out0, out1)
        return int(t.value)

    def sort(self, keys, rids, keys_out=None, rids_out=None, partitioner: str = "radix") -> int:
        keys_out = keys_out if keys_out is not None else _torch().empty_like(keys)
        rids_out = rids_out if rids_out is not None else _torch().empty_like(rids)
        return self._submit(TJ_OP_SORT, keys, rids, None, None, keys_out, rids_out, 0, partitioner)

    def join_count(self, r_keys, s_keys, partitioner: str = "radix") -> int:
        return self._submit(TJ_OP_JOIN_COUNT, r_keys, None, s_keys, None, None, None, 0, partitioner)

    def join(self, r_keys, r_rids, s_keys, s_rids, capacity: int, out_r=None, out_s=None,
             partitioner: str = "radix") -> int:
        torch = _torch()
        out_r = out_r if out_r is not None else torch.empty(max(capacity, 1), dtype=torch.int32, device=r_keys.device)
        out_s = out_s if out_s is not None else torch.empty(max(capacity, 1), dtype=torch.int32, device=r_keys.device)
        return self._submit(TJ_OP_JOIN_MATERIALIZE, r_keys, r_rids, s_keys, s_rids, out_r, out_s, capacity,
                            partitioner)

    def wait(self, ticket: int) -> dict:
        """Blocks until the request is done; returns its status, count, timings
        and (sort) keys / rids or (join) out_r / out_s tensors."""
        r = Result()
        _check(load().tj_server_wait(self._h, ticket, ctypes.byref(r)), "tj_server_wait")
        op, _, out0, out1 = self._keep.pop(ticket)
        out = {"status": r.status, "op": r.op, "count": int(r.count), "queue_ms": r.queue_ms, "run_ms": r.run_ms,
               "total_ms": r.total_ms, "learned": int(r.learned), "key_ranges": int(r.key_ranges),
               "fused": int(r.fused), "windows": int(r.windows)}
        if r.status == TJ_OK and op == TJ_OP_SORT:
            out["keys"], out["rids"] = out0, out1
        elif r.status == TJ_OK and op == TJ_OP_JOIN_MATERIALIZE:
            out["out_r"], out["out_s"] = out0[:r.count], out1[:r.count]
        return out

    def configure(self, fuse_max_rows: int, fuse_max_requests: int = 32) -> None:
        """tj_server_configure: fuse requests of at most fuse_max_rows rows,
        at most fuse_max_requests per call (fuse_max_rows = 0: no fusion)."""
        _check(load().tj_server_configure(self._h, fuse_max_rows, fuse_max_requests), "tj_server_configure")

    def memory(self):
        """(arena bytes reserved now, peak so far)."""
        a, b = _u64(), _u64()
        _check(load().tj_server_memory(self._h, ctypes.byref(a), ctypes.byref(b)), "tj_server_memory")
        return int(a.value), int(b.value)

    def close(self) -> None:
        if self._h:
            _check(load().tj_server_destroy(self._h), "tj_server_destroy")
            self._h = _P()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

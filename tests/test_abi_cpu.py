"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function the header declares, reports workspace sizes, and rejects bad
arguments before issuing any device work."""
import ctypes
import os
import re

import pytest

from paper_2602_21237_amd import tj

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tj.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tj_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    lib = tj.load()
    names = _declared()
    assert "tj_sort" in names and "tj_join_count" in names and "tj_join_materialize" in names
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(tj.EXPORTS), "binding and header disagree"


def test_version_and_strerror():
    assert tj.load().tj_version() >= 100
    for s in (0, -1, -2, -3, -4, -5, -6, -7):
        assert tj.strerror(s) and tj.strerror(s) != "unknown status"


@pytest.mark.parametrize("op", [tj.TJ_OP_SORT, tj.TJ_OP_JOIN_COUNT, tj.TJ_OP_JOIN_MATERIALIZE])
def test_workspace_query(op):
    mn, full = tj.workspace_query(op, tj.TJ_KEY_I64, 1_000_000, 1_000_000)
    assert 0 < mn <= (1 << 20) < full  # a 1 MiB budget is accepted
    mn2, full2 = tj.workspace_query(op, tj.TJ_KEY_I64, 2_000_000, 2_000_000)
    assert mn2 == mn and full2 > full  # minimum is size independent, full grows
    row = 12 if op != tj.TJ_OP_JOIN_COUNT else 8
    nbuf = 1 if op == tj.TJ_OP_SORT else 4
    assert full - full2 // 2 < full and full >= nbuf * row * 1_000_000 // (2 if op == 0 else 1) // 2


def test_workspace_query_errors():
    lib = tj.load()
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    assert lib.tj_workspace_query(0, 3, 10, 0, ctypes.byref(a), ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_workspace_query(7, 8, 10, 0, ctypes.byref(a), ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_workspace_query(1, 8, 1 << 31, 5, ctypes.byref(a), ctypes.byref(b)) == tj.TJ_E_TOO_LARGE
    assert lib.tj_workspace_query(1, 8, 10, 5, None, ctypes.byref(b)) == tj.TJ_E_ARG


# Fake, never dereferenced device addresses: the checks below all fail before
# the library touches the device.
A, B, C, D, W = 0x10000000, 0x20000000, 0x30000000, 0x40000000, 0x50000000


def test_sort_argument_errors():
    lib = tj.load()
    n = 1000
    assert lib.tj_sort(5, A, B, n, C, D, W, 1 << 30, None, None) == tj.TJ_E_ARG
    assert lib.tj_sort(8, A, B, 1 << 31, C, D, W, 1 << 30, None, None) == tj.TJ_E_TOO_LARGE
    assert lib.tj_sort(8, None, B, n, C, D, W, 1 << 30, None, None) == tj.TJ_E_ARG
    assert lib.tj_sort(8, A, B, n, C, D, W + 8, 1 << 30, None, None) == tj.TJ_E_WORKSPACE
    assert lib.tj_sort(8, A, B, n, A + 8, D, W, 1 << 30, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_sort(8, A, B, n, C, C + 4000, W, 1 << 30, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_sort(8, A, B, n, C, D, C + 256, 1 << 30, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_sort(8, A, B, n, C, D, W, 1024, None, None) == tj.TJ_E_WORKSPACE
    assert lib.tj_sort(8, A, B, 0, C, D, W, 0, None, None) == tj.TJ_OK  # empty input: no work


def test_join_argument_errors():
    lib = tj.load()
    cnt = ctypes.c_uint64(7)
    assert lib.tj_join_count(8, A, 10, B, 10, None, W, 1 << 30, None, None) == tj.TJ_E_ARG
    assert lib.tj_join_count(4, A, 1 << 31, B, 10, ctypes.byref(cnt), W, 1 << 30, None, None) == tj.TJ_E_TOO_LARGE
    assert lib.tj_join_count(8, A, 0, B, 10, ctypes.byref(cnt), W, 1 << 30, None, None) == tj.TJ_OK
    assert cnt.value == 0
    assert lib.tj_join_count(8, A, 10, B, 10, ctypes.byref(cnt), W, 100, None, None) == tj.TJ_E_WORKSPACE
    assert lib.tj_join_materialize(8, A, None, 10, B, D, 10, C, W, 100, ctypes.byref(cnt), 0x60000000,
                                   1 << 30, None, None) == tj.TJ_E_ARG
    # out_r overlapping an input
    assert lib.tj_join_materialize(8, A, B, 10, C, D, 10, A, W, 100, ctypes.byref(cnt), 0x60000000,
                                   1 << 30, None, None) == tj.TJ_E_ALIAS
    # out_r overlapping out_s
    assert lib.tj_join_materialize(8, A, B, 10, C, D, 10, W, W + 40, 100, ctypes.byref(cnt), 0x60000000,
                                   1 << 30, None, None) == tj.TJ_E_ALIAS


def test_workspace_overlapping_an_input():
    lib = tj.load()
    n = 1000
    cnt = ctypes.c_uint64(0)
    # the workspace over the sort's keys or rids
    assert lib.tj_sort(8, A, B, n, C, D, A + 256, 1 << 20, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_sort(8, A, B, n, C, D, B - 256, 1 << 20, None, None) == tj.TJ_E_ALIAS
    # the workspace over a join's key or rid columns
    assert lib.tj_join_count(8, A, n, B, n, ctypes.byref(cnt), B - 256, 1 << 20, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_join_materialize(8, A, B, n, C, D, n, 0x60000000, 0x61000000, 10, ctypes.byref(cnt),
                                   D + 256, 1 << 20, None, None) == tj.TJ_E_ALIAS
    # the path selector's workspace over a key column
    need = ctypes.c_uint64()
    assert lib.tj_select_workspace_query(n, n, ctypes.byref(need)) == tj.TJ_OK
    out = tj.Selection()
    assert lib.tj_select_path(tj.TJ_OP_JOIN_COUNT, 8, A, n, B, n, None, ctypes.byref(out), None, A,
                              need.value, None) == tj.TJ_E_ALIAS
    # composite keys: the workspace over a key column or the rids
    two = (ctypes.c_int * 2)(8, 4)
    cols = (ctypes.c_void_p * 2)(A, B)
    outs = (ctypes.c_void_p * 2)(C, C + 8000)
    assert lib.tj_sort_multi(2, two, cols, D, n, outs, W, B, 1 << 20, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_join_count_multi(2, two, cols, n, cols, n, ctypes.byref(cnt), A + 4096, 1 << 20, None,
                                   None) == tj.TJ_E_ALIAS


def test_host_allocation_failure_returns_internal():
    """A host allocation that throws inside the planner comes back as
    TJ_E_INTERNAL (no C++ exception crosses the C ABI). The self-test flag
    makes the first host allocation of every sort and join call fail before
    any device work, so fake device addresses are never touched."""
    lib = tj.load()
    n = 1000
    cnt = ctypes.c_uint64(0)
    opt = tj.Options(tj.TJ_PART_LEARNED, 0, 0)
    m = tj.RmiModel()
    tj.debug_set_flags(tj.TJ_DEBUG_FAIL_HOST_ALLOC)
    try:
        assert lib.tj_sort(8, A, B, n, C, D, W, 1 << 30, None, None) == tj.TJ_E_INTERNAL
        assert lib.tj_sort_ex(4, A, B, n, C, D, W, 1 << 30, None, ctypes.byref(opt), None) == tj.TJ_E_INTERNAL
        assert lib.tj_join_count(8, A, n, B, n, ctypes.byref(cnt), W, 1 << 30, None, None) == tj.TJ_E_INTERNAL
        assert lib.tj_join_count_ex(8, A, n, B, n, ctypes.byref(cnt), W, 1 << 30, None, ctypes.byref(opt),
                                    None) == tj.TJ_E_INTERNAL
        assert lib.tj_join_materialize(8, A, B, n, C, D, n, 0x60000000, 0x61000000, 10, ctypes.byref(cnt),
                                       W, 1 << 26, None, None) == tj.TJ_E_INTERNAL
        assert lib.tj_rmi_train(8, A, n, None, 0, 0, ctypes.byref(m), W, 1 << 30, None) == tj.TJ_E_INTERNAL
        assert lib.tj_debug_partition_pass(A, B, n, 0, 0, 8, 0, C, D, 0x60000000, W, 1 << 30,
                                           None) == tj.TJ_E_INTERNAL
        # argument errors are still found first
        assert lib.tj_sort(8, None, B, n, C, D, W, 1 << 30, None, None) == tj.TJ_E_ARG
    finally:
        tj.debug_set_flags(0)
    assert lib.tj_debug_set_flags(8) == tj.TJ_E_ARG


def _c_sizeof(type_name: str) -> int:
    import subprocess
    import tempfile
    src = '#include <stdio.h>\n#include "tj.h"\nint main(void){printf("%%zu", sizeof(%s));return 0;}\n' % type_name
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "s.c"), os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        return int(subprocess.check_output([exe]).decode())


def test_struct_layouts_match_header():
    assert ctypes.sizeof(tj.Stats) == _c_sizeof("tj_stats_t")
    assert ctypes.sizeof(tj.Options) == _c_sizeof("tj_options_t")
    assert ctypes.sizeof(tj.RmiModel) == _c_sizeof("tj_rmi_t")


def test_learned_option_errors():
    lib = tj.load()
    bad = tj.Options(7, 0, 0)
    assert lib.tj_sort_ex(8, A, B, 1000, C, D, W, 1 << 30, None, ctypes.byref(bad), None) == tj.TJ_E_ARG
    bad = tj.Options(tj.TJ_PART_LEARNED, 1001, 0)
    cnt = ctypes.c_uint64(0)
    assert lib.tj_join_count_ex(8, A, 10, B, 10, ctypes.byref(cnt), W, 1 << 30, None, ctypes.byref(bad),
                                None) == tj.TJ_E_ARG
    ok = tj.Options(tj.TJ_PART_LEARNED, 0, 0)
    assert lib.tj_sort_ex(8, A, B, 0, C, D, W, 0, None, ctypes.byref(ok), None) == tj.TJ_OK  # empty input
    assert lib.tj_sort_ex(8, A, B, 1 << 31, C, D, W, 1 << 30, None, ctypes.byref(ok), None) == tj.TJ_E_TOO_LARGE


def test_rmi_entry_point_errors():
    lib = tj.load()
    b = ctypes.c_uint64(0)
    assert lib.tj_rmi_workspace_query(8, 0, 0, 0, ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_rmi_workspace_query(3, 10, 0, 0, ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_rmi_workspace_query(8, 1 << 31, 0, 0, ctypes.byref(b)) == tj.TJ_E_TOO_LARGE
    assert lib.tj_rmi_workspace_query(8, 1 << 20, 1 << 20, 10, ctypes.byref(b)) == tj.TJ_OK
    assert b.value > ctypes.sizeof(tj.RmiModel) + 2 * 20972 * 12
    m = tj.RmiModel()
    assert lib.tj_rmi_train(8, None, 10, None, 0, 0, ctypes.byref(m), W, 1 << 30, None) == tj.TJ_E_ARG
    assert lib.tj_rmi_train(8, A, 10, None, 5, 0, ctypes.byref(m), W, 1 << 30, None) == tj.TJ_E_ARG
    assert lib.tj_rmi_train(8, A, 1000, None, 0, 0, ctypes.byref(m), W, 4096, None) == tj.TJ_E_WORKSPACE
    # models that would break monotonicity or the bucket range are refused before device work
    good = _valid_model()
    assert lib.tj_rmi_buckets(8, A, 0, ctypes.byref(good), C, W, 1 << 20, None) == tj.TJ_OK
    for field, idx, val in (("buckets", None, 0), ("buckets", None, 513), ("knot", 5, 0),
                            ("leaf_hi", 3, 600), ("leaf_lo", 4, 0), ("leaf_b", 9, -1.0),
                            ("knot_inv", 2, float("inf"))):
        bad = _valid_model()
        if idx is None:
            setattr(bad, field, val)
        else:
            getattr(bad, field)[idx] = val
        assert lib.tj_rmi_buckets(8, A, 100, ctypes.byref(bad), C, W, 1 << 20, None) == tj.TJ_E_ARG, field


def _valid_model():
    m = tj.RmiModel()
    m.buckets = 512
    for i in range(tj.RMI_SEGMENTS + 1):
        m.knot[i] = 1000 * i
    for i in range(tj.RMI_SEGMENTS):
        m.knot_inv[i] = 1.0 / 1000
    for l in range(tj.RMI_LEAVES):
        m.leaf_lo[l] = m.leaf_hi[l] = l // 2
    return m


def test_server_argument_errors():
    lib = tj.load()
    h = ctypes.c_void_p()
    assert lib.tj_server_create(None, 1 << 30, 4, ctypes.byref(h)) == tj.TJ_E_ARG
    assert lib.tj_server_create(W, 1 << 30, 0, ctypes.byref(h)) == tj.TJ_E_ARG
    assert lib.tj_server_create(W, 1 << 30, 65, ctypes.byref(h)) == tj.TJ_E_ARG
    assert lib.tj_server_create(W + 8, 1 << 30, 4, ctypes.byref(h)) == tj.TJ_E_WORKSPACE
    assert lib.tj_server_create(W, 1000, 4, ctypes.byref(h)) == tj.TJ_E_WORKSPACE
    t = ctypes.c_uint64()
    req = tj.Request(tj.TJ_OP_SORT, 8, A, B, 10, None, None, 0, C, D, 0, 0, 0)
    assert lib.tj_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == tj.TJ_E_ARG
    assert lib.tj_server_wait(None, 1, ctypes.byref(tj.Result())) == tj.TJ_E_ARG
    assert lib.tj_server_destroy(None) == tj.TJ_E_ARG
    assert ctypes.sizeof(tj.Request) == _c_sizeof("tj_request_t")
    assert ctypes.sizeof(tj.Result) == _c_sizeof("tj_result_t")


def test_multi_argument_errors():
    lib = tj.load()
    two = (ctypes.c_int * 2)(8, 4)
    bad = (ctypes.c_int * 2)(8, 5)
    cols = (ctypes.c_void_p * 2)(A, B)
    outs = (ctypes.c_void_p * 2)(C, C + 8000)
    b = ctypes.c_uint64()
    assert lib.tj_multi_workspace_query(0, 0, two, 10, 0, ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_multi_workspace_query(0, 9, two, 10, 0, ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_multi_workspace_query(0, 2, bad, 10, 0, ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_multi_workspace_query(3, 2, two, 10, 0, ctypes.byref(b)) == tj.TJ_E_ARG
    assert lib.tj_multi_workspace_query(2, 2, two, 1 << 30, 1 << 30, ctypes.byref(b)) == tj.TJ_E_TOO_LARGE
    assert lib.tj_multi_workspace_query(0, 2, two, 1000, 0, ctypes.byref(b)) == tj.TJ_OK and b.value > 24000
    n = 1000
    assert lib.tj_sort_multi(2, bad, cols, D, n, outs, W, W + (1 << 20), 1 << 30, None, None) == tj.TJ_E_ARG
    assert lib.tj_sort_multi(2, two, cols, D, 1 << 31, outs, W, W + (1 << 20), 1 << 30, None, None) == tj.TJ_E_TOO_LARGE
    assert lib.tj_sort_multi(2, two, None, D, n, outs, W, W + (1 << 20), 1 << 30, None, None) == tj.TJ_E_ARG
    assert lib.tj_sort_multi(2, two, cols, D, n, outs, W, W + 8 + (1 << 20), 1 << 30, None, None) == tj.TJ_E_WORKSPACE
    aliased = (ctypes.c_void_p * 2)(A + 8, C + 8000)
    assert lib.tj_sort_multi(2, two, cols, D, n, aliased, W, W + (1 << 20), 1 << 30, None, None) == tj.TJ_E_ALIAS
    assert lib.tj_sort_multi(2, two, cols, D, 0, outs, W, W + (1 << 20), 1 << 30, None, None) == tj.TJ_OK
    cnt = ctypes.c_uint64(5)
    assert lib.tj_join_count_multi(2, two, cols, 10, cols, 10, None, W, 1 << 30, None, None) == tj.TJ_E_ARG
    assert lib.tj_join_count_multi(2, two, cols, 0, cols, 10, ctypes.byref(cnt), W, 1 << 30, None, None) == tj.TJ_OK
    assert cnt.value == 0


def test_select_argument_errors():
    lib = tj.load()
    assert ctypes.sizeof(tj.Selection) == _c_sizeof("tj_selection_t")
    assert ctypes.sizeof(tj.SelectOptions) == _c_sizeof("tj_select_options_t")
    b = ctypes.c_uint64()
    assert lib.tj_select_workspace_query(10, 10, None) == tj.TJ_E_ARG
    assert lib.tj_select_workspace_query(1 << 31, 0, ctypes.byref(b)) == tj.TJ_E_TOO_LARGE
    assert lib.tj_select_workspace_query(1 << 20, 1 << 20, ctypes.byref(b)) == tj.TJ_OK
    need = b.value
    assert need % 256 == 0 and need >= 2 * 64 * 16384 + 3 * 16384  # 64 blocks of 16384 rows per column
    out = tj.Selection()
    o = ctypes.byref(out)
    sel = lib.tj_select_path
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, B, 100, None, None, None, W, need, None) == tj.TJ_E_ARG
    assert sel(tj.TJ_OP_JOIN_COUNT, 5, A, 100, B, 100, None, o, None, W, need, None) == tj.TJ_E_ARG
    assert sel(7, 8, A, 100, B, 100, None, o, None, W, need, None) == tj.TJ_E_ARG
    assert sel(tj.TJ_OP_SORT, 8, A, 100, B, 100, None, o, None, W, need, None) == tj.TJ_E_ARG  # sort with n_s
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, None, 100, B, 100, None, o, None, W, need, None) == tj.TJ_E_ARG
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, None, 100, None, o, None, W, need, None) == tj.TJ_E_ARG
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 1 << 31, B, 100, None, o, None, W, need, None) == tj.TJ_E_TOO_LARGE
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, B, 100, None, o, None, W, 1000, None) == tj.TJ_E_WORKSPACE
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, B, 100, None, o, None, W + 8, need, None) == tj.TJ_E_WORKSPACE
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, B, 100, None, o, None, None, need, None) == tj.TJ_E_WORKSPACE
    # registers overlapping an input or the workspace
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, B, 100, None, o, A + 8, W, need, None) == tj.TJ_E_ALIAS
    assert sel(tj.TJ_OP_JOIN_COUNT, 8, A, 100, B, 100, None, o, W + 256, W, need, None) == tj.TJ_E_ALIAS


def test_stream_copy_argument_errors():
    lib = tj.load()
    cp = lib.tj_debug_stream_copy
    assert cp(None, B, 64, None) == tj.TJ_E_ARG
    assert cp(A, None, 64, None) == tj.TJ_E_ARG
    assert cp(A, B, 60, None) == tj.TJ_E_ARG  # not a multiple of 16 bytes
    assert cp(A + 8, B, 64, None) == tj.TJ_E_ARG  # misaligned
    assert cp(A, A + 32, 64, None) == tj.TJ_E_ALIAS


def _header_define(name):
    m = re.search(r"#define\s+%s\s+\(1ull << (\d+)\)" % name, open(HEADER).read())
    return 1 << int(m.group(1))


def test_select_defaults_match_header():
    assert tj.TJ_SELECT_DEFAULT_MIN_ROWS == _header_define("TJ_SELECT_DEFAULT_MIN_ROWS")
    assert tj.TJ_SELECT_DEFAULT_MIN_OUTPUT == _header_define("TJ_SELECT_DEFAULT_MIN_OUTPUT")

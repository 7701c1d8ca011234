"""MI355X-native tensor-path equi-join and sort (gfx950 HIP kernels behind a C ABI).

The library itself is lib/libtj.so (include/tj.h); this package is its thin
binding. Loading is lazy, and there is no CPU fallback: the calls raise when
the library is missing or no GPU is visible.
"""
from .tj import (TjError, join, join_count, load, sort, strerror, timing, timing_read,  # noqa: F401
                 workspace_query, sort_static, rmi_train, rmi_buckets, rmi_workspace_query, RmiModel, sort_multi,
                 join_count_multi, join_multi, multi_workspace_query,
                 select_path, select_workspace_query, TJ_PATH_LINEAR, TJ_PATH_TENSOR, debug_stream_copy,
                 TJ_SELECT_DEFAULT_MIN_ROWS, TJ_SELECT_DEFAULT_MIN_OUTPUT,
                 TJ_KEY_I32, TJ_KEY_I64, TJ_OP_SORT, TJ_OP_JOIN_COUNT, TJ_OP_JOIN_MATERIALIZE)

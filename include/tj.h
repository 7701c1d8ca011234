/*
 * tj.h - tensor-path equi-join and sort on one MI355X (gfx950).
 *
 * The paper's tensor-based execution path (Sec. III-IV) keeps relations as
 * columns ("a relation is a sparse set of coordinates, one axis per attribute",
 * Sec. III.B) and delays linearisation and materialisation to the last step
 * (Sec. III.A). Here a relation is two device columns, keys[n] and rids[n],
 * and the only materialised join output is the final (rid_R, rid_S) pairs.
 *
 * Every call takes a caller-owned device workspace of `workspace_bytes`; it
 * plays the role of the paper's work_mem budget M (Sec. VI, Eq. 1). Results
 * are identical for every budget >= the minimum reported by
 * tj_workspace_query; a smaller budget only costs extra passes over the inputs
 * (the GPU analogue of the spill term alpha(N, M)).
 *
 * Conventions shared by all calls:
 *   - key_type: TJ_KEY_I32 (int32_t keys) or TJ_KEY_I64 (int64_t keys). Keys
 *     are compared as signed integers.
 *   - All array pointers are device pointers into caller-owned memory. Inputs
 *     are read-only; outputs must not overlap inputs or the workspace
 *     (TJ_E_ALIAS). The library allocates no device memory.
 *   - workspace: device memory of workspace_bytes bytes, 256-byte aligned.
 *     Its contents are undefined after a call.
 *   - stream: a hipStream_t (NULL = the null stream). Work is ordered on it.
 *     Each call returns after its results are complete on `stream` (the
 *     planner reads small tables back between passes).
 *   - Row counts must be < 2^31 (row ids and positions are int32): larger
 *     values give TJ_E_TOO_LARGE.
 *   - Argument errors are reported before any device work is issued.
 *   - stats (may be NULL) receives the plan's bookkeeping (tj_stats_t).
 *   - Calls on different streams from different host threads may overlap.
 */
#ifndef TJ_H
#define TJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum tj_key_type { TJ_KEY_I32 = 4, TJ_KEY_I64 = 8 };

enum tj_op { TJ_OP_SORT = 0, TJ_OP_JOIN_COUNT = 1, TJ_OP_JOIN_MATERIALIZE = 2 };

enum tj_status {
    TJ_OK = 0,
    TJ_E_ARG = -1,        /* NULL pointer where one is required, bad key type or op */
    TJ_E_WORKSPACE = -2,  /* workspace_bytes below the minimum, or misaligned */
    TJ_E_CAPACITY = -3,   /* join result larger than `capacity` (count still set) */
    TJ_E_TOO_LARGE = -4,  /* a row count >= 2^31 */
    TJ_E_ALIAS = -5,      /* an output overlaps an input or the workspace */
    TJ_E_HIP = -6,        /* a HIP runtime call or kernel launch failed */
    TJ_E_INTERNAL = -7    /* a planner invariant failed (a library bug) */
};

/* Plan bookkeeping of one call. Byte counts are the algorithmic HBM bytes of
 * the executed plan (each kernel's reads and writes of row data), not
 * hardware counters. */
typedef struct {
    uint64_t bytes_read;
    uint64_t bytes_written;
    uint64_t workspace_used;  /* peak workspace bytes the plan touched */
    uint32_t passes;          /* partition passes (histogram + scan + scatter) */
    uint32_t leaves;          /* per-bucket LDS sort / join blocks */
    uint32_t single_key;      /* buckets holding a single key value */
    uint32_t key_ranges;      /* key ranges processed one at a time (1 = budget not binding) */
} tj_stats_t;

/*
 * Workspace sizes for an operation.
 *   op:        TJ_OP_SORT (n_r = rows, n_s ignored), TJ_OP_JOIN_COUNT or
 *              TJ_OP_JOIN_MATERIALIZE (n_r, n_s = rows of R and S).
 *   min_bytes: smallest workspace any call of this shape accepts.
 *   full_bytes: workspace at which the budget never binds (one key range).
 * Host-only; issues no device work. Returns TJ_OK, TJ_E_ARG or TJ_E_TOO_LARGE.
 */
int tj_workspace_query(int op, int key_type, uint64_t n_r, uint64_t n_s,
                       uint64_t *min_bytes, uint64_t *full_bytes);

/*
 * Tensor-based sort (Sec. IV.B): relocate the rows along the key axis.
 * Writes the stable ascending order of (keys_in, rids_in) by signed key:
 *   keys_out[i] = keys_in[p(i)], rids_out[i] = rids_in[p(i)], where p is the
 *   unique permutation with keys ascending and, among equal keys, input
 *   positions ascending.
 *   keys_in [n] (int32 or int64 per key_type), rids_in [n] int32: inputs.
 *   keys_out[n], rids_out[n]: outputs (device, caller-owned, no overlap).
 * n = 0 is allowed and does nothing.
 */
int tj_sort(int key_type, const void *keys_in, const int32_t *rids_in, uint64_t n,
            void *keys_out, int32_t *rids_out,
            void *workspace, uint64_t workspace_bytes, void *stream, tj_stats_t *stats);

/*
 * Tensor-based hash join, count only (Sec. IV.A): the inner equi-join size
 *   |R join S| = sum over key values k of cnt_R(k) * cnt_S(k),
 * written to *count (host pointer) as an unsigned 64-bit integer.
 *   r_keys[n_r], s_keys[n_s]: device key columns of R and S (same key_type).
 */
int tj_join_count(int key_type, const void *r_keys, uint64_t n_r,
                  const void *s_keys, uint64_t n_s, uint64_t *count,
                  void *workspace, uint64_t workspace_bytes, void *stream, tj_stats_t *stats);

/*
 * Tensor-based hash join with late materialisation (Sec. IV.A, Sec. III.A):
 * the keys of R and S are aligned on the common key axis and only the final
 * (rid_R, rid_S) pairs are written, in canonical order:
 *   ascending key, then R input position, then S input position
 *   (for one key: R row i1 with every matching S row in S order, then R row i2 ...).
 *   r_keys[n_r], r_rids[n_r], s_keys[n_s], s_rids[n_s]: device inputs.
 *   out_r[capacity], out_s[capacity]: device outputs; pair t is
 *     (out_r[t], out_s[t]).
 *   *count (host): set to |R join S| on TJ_OK and on TJ_E_CAPACITY.
 * If |R join S| > capacity the call returns TJ_E_CAPACITY; the contents of
 * out_r/out_s are then unspecified, and no element at or beyond `capacity`
 * is ever written.
 */
int tj_join_materialize(int key_type, const void *r_keys, const int32_t *r_rids, uint64_t n_r,
                        const void *s_keys, const int32_t *s_rids, uint64_t n_s,
                        int32_t *out_r, int32_t *out_s, uint64_t capacity, uint64_t *count,
                        void *workspace, uint64_t workspace_bytes, void *stream, tj_stats_t *stats);

/*
 * Per-kernel timing (profiling hook). tj_timing(1) clears the counters and
 * makes every later call record a HIP event pair around each kernel launch on
 * the call's stream; tj_timing(0) stops recording. tj_timing_read copies up to
 * `max` entries, one per kernel family, and returns the number written.
 *   launches: kernel dispatches of the family;
 *   bytes:    algorithmic bytes those dispatches move (row data read and
 *             written, as planned: not hardware counters);
 *   ms:       summed event-measured durations.
 * Timing is process-wide and guarded by a mutex; it adds two event records
 * per launch.
 */
typedef struct {
    char name[24];
    uint64_t launches;
    uint64_t bytes;
    double ms;
} tj_kernel_stat_t;

int tj_timing(int enable);
int tj_timing_read(tj_kernel_stat_t *out, int max);

/* Static text for a status code. */
const char *tj_strerror(int status);

/* Library version as major*10000 + minor*100 + patch. */
int tj_version(void);

/*
 * Kernel self-test hooks used by the per-kernel parity tests.
 *
 * tj_debug_wave_scan: inclusive prefix sum of `in` within each 64-lane
 *   wavefront (n values, n a multiple of 64), written to `out`. Exercises the
 *   DPP scan primitive every offset computation is built on.
 * tj_debug_partition_pass: one stable radix partition pass over n int64 keys
 *   (with int32 rids): digit(k) = ((ord(k) - base) >> shift) & (2^bits - 1)
 *   with ord the order-preserving map of signed keys to unsigned, rows written
 *   to keys_out/rids_out grouped by digit ascending, input order kept within a
 *   digit; counts_out[2^bits] (device, uint32) receives the digit histogram.
 *   bits in [1, 9]; base must be <= every ord(k); shift + bits <= 64.
 *   flags: 0, or TJ_DEBUG_FORCE_REORDER to make every scatter tile take the
 *   path that re-ranks it when its first ranking is not in input order (the
 *   result must not change). Other bits give TJ_E_ARG.
 */
#define TJ_DEBUG_FORCE_REORDER 1u
/*
 * tj_debug_set_flags: process-wide self-test switch for every later call.
 *   TJ_DEBUG_FORCE_REORDER: each partition tile and each join block also runs
 *   the ballot-ranked path that replaces an atomic-ranked order found out of
 *   input order; results must not change, only time. 0 turns it off.
 *   Returns TJ_OK, or TJ_E_ARG for unknown bits.
 */
int tj_debug_set_flags(uint32_t flags);
int tj_debug_wave_scan(const uint32_t *in, uint32_t *out, uint64_t n, void *stream);
int tj_debug_partition_pass(const int64_t *keys, const int32_t *rids, uint64_t n,
                            uint64_t base, uint32_t shift, uint32_t bits, uint32_t flags,
                            int64_t *keys_out, int32_t *rids_out, uint32_t *counts_out,
                            void *workspace, uint64_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TJ_H */

/*
 * tj.h - tensor-path equi-join and sort on one MI355X (gfx950).
 *
 * The paper's tensor-based execution path (Sec. III-IV) keeps relations as
 * columns: a relation is treated as a sparse set of points with one coordinate
 * axis per attribute (Sec. III.B), and linearisation and materialisation are
 * delayed to the last step (Sec. III.A). Here a relation is two device
 * columns, keys[n] and rids[n], and the only materialised join output is the
 * final (rid_R, rid_S) pairs.
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
 *     are read-only; outputs must not overlap inputs or the workspace, and the
 *     workspace must not overlap an input (TJ_E_ALIAS). No call allocates
 *     device memory (tj_sort_static works in a fixed array that the library's
 *     code object brings with it).
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
    TJ_E_ALIAS = -5,      /* an output overlaps an input or the workspace, or the workspace an input */
    TJ_E_HIP = -6,        /* a HIP runtime call or kernel launch failed */
    TJ_E_INTERNAL = -7    /* a planner invariant failed (a library bug), or host memory ran out */
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
    uint32_t key_ranges;      /* key ranges processed one at a time, each read from the
                                 inputs (1 = the inputs are read once) */
    uint32_t learned;         /* 1 when the first pass used the learned bucket function */
    uint32_t learned_overflow;/* buckets of that pass holding more than twice the mean */
    uint32_t windows;         /* under a binding budget, runs of buckets taken through the
                                 workspace window (sort), or key ranges whose buckets took
                                 further passes there (join); 0 when it does not bind */
    uint32_t pivots;          /* crowded buckets split three ways around a sampled frequent
                                 key (below, equal, above) instead of by a radix digit */
    uint64_t sample_rows;     /* keys the learned model was fitted to */
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
 * A bucket crowded by one frequent key (it holds more than twice the rows
 * its parent's digit gave each bucket, and three sampled rows mostly agree
 * on a key) is split below / equal / above that key in its next unfiltered
 * pass instead of by a radix digit (tj_stats_t.pivots); the output does not
 * depend on it.
 * Under a binding budget (workspace_bytes below tj_workspace_query's
 * full_bytes) the first partition pass still reads the input once and writes
 * every row into keys_out/rids_out, where leaf buckets are then sorted in
 * place. Buckets that need more passes take them through the workspace, as
 * many adjacent buckets at a time as it holds (tj_stats_t.windows counts those
 * runs). A bucket larger than the workspace that holds more than one key value
 * is sorted the same way into its own rows of the output, from the input read
 * again and filtered to the bucket's key range (key_ranges - 1 such reads).
 */
int tj_sort(int key_type, const void *keys_in, const int32_t *rids_in, uint64_t n,
            void *keys_out, int32_t *rids_out,
            void *workspace, uint64_t workspace_bytes, void *stream, tj_stats_t *stats);

/*
 * tj_sort for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, semantics, results and errors as tj_sort, without the
 * workspace: the call uses a device array of TJ_STATIC_SCRATCH_BYTES (256 MiB)
 * that the library holds on every GPU it runs on, from the library's load
 * until the process ends, as its workspace budget. Inputs of up to 22,346,560
 * int64 rows (33,519,872 int32 rows) run the unlimited plan; larger ones run
 * the budget-bound plan (the array as the window of tj_sort under a binding
 * budget), so results never change, only time.
 * The call makes no device or pinned-host allocation (its read-backs go to
 * grow-only pageable host memory) and records no timing events.
 * The array is shared by every call on one GPU: the library serialises those
 * calls (each returns after its work is complete on `stream`), so two calls
 * on one GPU never overlap; nothing is carried from one call to the next.
 * `stream` must belong to the current device.
 * Errors: as tj_sort; TJ_E_WORKSPACE if the shape's minimum workspace exceeds
 * the array (no row count below 2^31 does); TJ_E_HIP if the array's device
 * address cannot be obtained.
 */
#define TJ_STATIC_SCRATCH_BYTES (256ull << 20)
int tj_sort_static(int key_type, const void *keys_in, const int32_t *rids_in, uint64_t n,
                   void *keys_out, int32_t *rids_out, void *stream, tj_stats_t *stats);

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
 * Learned CDF partitioner.
 *
 * The paper lets what the execution stage observes about the data decide how
 * the tensor path runs (Sec. III.C). Here that observation is a sample of the
 * keys, and what it decides is the bucket function of the first partition
 * pass: a two-layer recursive model index (RMI) that estimates each key's
 * rank replaces the radix digit, so that buckets hold similar row counts even
 * for skewed key distributions, where radix digits over the key range leave
 * most rows in a few buckets and need extra passes. Later passes use radix
 * digits over each bucket's own key range (a bucket is never split by the
 * model again), and the leaf sorts and joins are unchanged, so results are
 * bit-identical to the radix path: the bucket function only has to be
 * non-decreasing in the key, which the model guarantees by construction.
 *
 * Model (all keys as ordinals: ord(k) = k XOR 2^63 for int64, k XOR 2^31 for
 * int32, as unsigned; every float operation is one IEEE f32 operation rounded
 * to nearest even, never fused):
 *   root:   j = the largest i in [0, TJ_RMI_SEGMENTS - 1] with i = 0 or
 *           knot[i] <= x; d = clamp(x, knot[j], knot[j+1]) - knot[j];
 *           t = f32(d) * knot_inv[j]; leaf = 4 j + min(floor(4 t), 3).
 *   leaf l: sd = x - leaf_base[l] as a signed integer saturated to +-2^62;
 *           y = leaf_a[l] + leaf_b[l] * f32(sd);
 *           bucket = floor(clamp(y, leaf_lo[l], leaf_hi[l])).
 * Training (tj_rmi_train, and the learned calls): a relation of n rows is
 * sampled at positions floor(i n / m), i < m = max(min(n, 2048),
 * n * permille / 1000); a join samples R and S and fits one model to the
 * union. The sample is sorted by the plain (radix) sort path. knot[i] is the
 * sorted sample's element floor(i (M - 1) / TJ_RMI_SEGMENTS) (M sample rows),
 * knot_inv[i] = f32(1 / f64(knot[i+1] - knot[i])) or 0 for equal knots. Each
 * leaf is fitted by least squares (fp64 sums) to its sample points with
 * targets F i / M (i = rank in the sample, F = buckets), slope clamped at 0;
 * leaf_lo/leaf_hi are the buckets of its first and last point, and a leaf
 * without points takes the next leaf's leaf_lo for both. Hence leaf_hi[l] <=
 * leaf_lo[l+1], which with slopes >= 0 makes the bucket non-decreasing in x.
 */
#define TJ_RMI_SEGMENTS 256
#define TJ_RMI_LEAVES 1024
typedef struct {
    uint64_t knot[TJ_RMI_SEGMENTS + 1];  /* key ordinals, non-decreasing */
    float knot_inv[TJ_RMI_SEGMENTS];
    uint64_t leaf_base[TJ_RMI_LEAVES];   /* key ordinal of each leaf's first sample point */
    float leaf_a[TJ_RMI_LEAVES];         /* intercept, in buckets */
    float leaf_b[TJ_RMI_LEAVES];         /* slope, in buckets per ordinal step (>= 0) */
    uint16_t leaf_lo[TJ_RMI_LEAVES];
    uint16_t leaf_hi[TJ_RMI_LEAVES];
    uint32_t buckets;                    /* F: buckets of the learned pass (512) */
    uint32_t sample_rows;                /* M */
} tj_rmi_t;

/*
 * TJ_PART_AUTO decides at execution time from the data, by the first radix
 * digit's bucket counts: if one bucket holds more than half of all rows, the
 * digit has not separated the bulk of the keys from a long tail (each radix
 * level narrows the digit to its bucket's key range, which splits a few dense
 * intervals at the next level but not a heavy tail), and the call trains the
 * learned model and partitions with it; otherwise it runs radix. Calls of at
 * least 2^22 rows with the full workspace count every 4096th key (the sample
 * their first digit range is taken from, read back to the host); smaller ones
 * count the first pass's histogram, before anything is moved.
 */
enum tj_partitioner { TJ_PART_RADIX = 0, TJ_PART_LEARNED = 1, TJ_PART_AUTO = 2 };
typedef struct {
    uint32_t partitioner;       /* TJ_PART_RADIX, TJ_PART_LEARNED or TJ_PART_AUTO */
    uint32_t sample_permille;   /* sample per relation in 1/1000 of its rows; 0 means 10 (1%) */
    uint64_t learned_min_rows;  /* rows (R + S) below which the radix digit is kept; 0 means 2^22.
                                   Values below 8193 act as 8193 (one LDS block holds smaller inputs) */
} tj_options_t;

/*
 * tj_sort_ex, tj_join_count_ex, tj_join_materialize_ex: tj_sort, tj_join_count
 * and tj_join_materialize with options (opt may be NULL: radix, as the plain
 * calls). TJ_PART_LEARNED applies when the workspace holds the full plan (at
 * least full_bytes of tj_workspace_query) and the call has at least
 * learned_min_rows rows; otherwise the call runs the radix path (stats.learned
 * tells which ran). The model is trained on the call's stream inside the
 * workspace; arguments, errors and results are those of the plain calls.
 * Unknown partitioner values give TJ_E_ARG.
 */
int tj_sort_ex(int key_type, const void *keys_in, const int32_t *rids_in, uint64_t n,
               void *keys_out, int32_t *rids_out, void *workspace, uint64_t workspace_bytes,
               void *stream, const tj_options_t *opt, tj_stats_t *stats);
int tj_join_count_ex(int key_type, const void *r_keys, uint64_t n_r, const void *s_keys, uint64_t n_s,
                     uint64_t *count, void *workspace, uint64_t workspace_bytes, void *stream,
                     const tj_options_t *opt, tj_stats_t *stats);
int tj_join_materialize_ex(int key_type, const void *r_keys, const int32_t *r_rids, uint64_t n_r,
                           const void *s_keys, const int32_t *s_rids, uint64_t n_s,
                           int32_t *out_r, int32_t *out_s, uint64_t capacity, uint64_t *count,
                           void *workspace, uint64_t workspace_bytes, void *stream,
                           const tj_options_t *opt, tj_stats_t *stats);

/*
 * tj_rmi_workspace_query: device workspace bytes tj_rmi_train needs for
 * relations of n_a and n_b rows (n_b = 0: one relation). Host only.
 * tj_rmi_train: fits the model to the sample of keys_a[n_a] and, when n_b > 0,
 * keys_b[n_b] (device key columns), on the GPU, and copies it to *model (host
 * memory). permille 0 means 10. Synchronises `stream` before returning.
 * Errors: TJ_E_ARG (bad key type, NULL pointers, n_a = 0), TJ_E_TOO_LARGE,
 * TJ_E_WORKSPACE (below the queried size or misaligned), TJ_E_HIP.
 */
int tj_rmi_workspace_query(int key_type, uint64_t n_a, uint64_t n_b, uint32_t permille, uint64_t *bytes);
int tj_rmi_train(int key_type, const void *keys_a, uint64_t n_a, const void *keys_b, uint64_t n_b,
                 uint32_t permille, tj_rmi_t *model, void *workspace, uint64_t workspace_bytes,
                 void *stream);
/*
 * tj_rmi_buckets: buckets[i] = bucket(ord(keys[i])) of the model *model (host
 * memory, copied to the workspace, which needs sizeof(tj_rmi_t) bytes,
 * 256-byte aligned) for n device keys, into the device array buckets[n].
 * The model must satisfy the layout rules above (knots non-decreasing,
 * 0 < buckets <= 512, leaf_lo <= leaf_hi < buckets): TJ_E_ARG otherwise.
 * Stream-ordered; returns without synchronising.
 */
int tj_rmi_buckets(int key_type, const void *keys, uint64_t n, const tj_rmi_t *model,
                   uint16_t *buckets, void *workspace, uint64_t workspace_bytes, void *stream);

/*
 * Composite (multi-column) keys.
 *
 * A relation keyed by m columns is a set of points in an m-dimensional key
 * space (Sec. III.B); the sort orders them lexicographically, column 0 first
 * (the row-major linearisation of that space), and the join matches rows
 * whose points coincide in every column (Sec. IV.A, a join condition over
 * several common attributes). Columns may mix int32 and int64 (signed); a
 * column's type must be the same in R and S.
 *
 * Method: the minimum and maximum of every column give its bit width b_c
 * (of max - min). Columns whose widths sum to at most 64 bits are packed
 * into one key (column minimum subtracted, most significant column first),
 * which orders and matches exactly like the tuple; the packed key is 4 bytes
 * when it fits 32 bits. Sort: one stable sort on the packed key, or, when
 * the widths exceed 64 bits, stable sorts on groups of columns of at most 64
 * bits each, least significant group first (LSD), carrying the permutation.
 * Join: one join on the packed keys; beyond 64 bits, R and S are sorted
 * together by their tuples, each distinct tuple is numbered in order (a
 * dense rank), and the join runs on the ranks. Results are those of the
 * single-key calls on the tuples: stable lexicographic order; canonical pair
 * order (tuple, then R position, then S position).
 *
 *   ncols: 1 .. TJ_MAX_KEY_COLS; key_types[c]: TJ_KEY_I32 or TJ_KEY_I64;
 *   keys_in[c] / r_keys[c] / s_keys[c]: device key columns;
 *   keys_out[c]: device output columns (same types), rids as in tj_sort.
 * Workspace: tj_multi_workspace_query gives the bytes at which no budget
 * binds; smaller workspaces are accepted down to the fixed arrays of the call
 * plus the minimum of its inner sort or join (TJ_E_WORKSPACE below that).
 * Errors as for the single-key calls; outputs must not overlap inputs or the
 * workspace (TJ_E_ALIAS).
 */
#define TJ_MAX_KEY_COLS 8
int tj_multi_workspace_query(int op, int ncols, const int *key_types, uint64_t n_r, uint64_t n_s,
                             uint64_t *bytes);
int tj_sort_multi(int ncols, const int *key_types, const void *const *keys_in, const int32_t *rids_in,
                  uint64_t n, void *const *keys_out, int32_t *rids_out, void *workspace,
                  uint64_t workspace_bytes, void *stream, tj_stats_t *stats);
int tj_join_count_multi(int ncols, const int *key_types, const void *const *r_keys, uint64_t n_r,
                        const void *const *s_keys, uint64_t n_s, uint64_t *count, void *workspace,
                        uint64_t workspace_bytes, void *stream, tj_stats_t *stats);
int tj_join_materialize_multi(int ncols, const int *key_types, const void *const *r_keys,
                              const int32_t *r_rids, uint64_t n_r, const void *const *s_keys,
                              const int32_t *s_rids, uint64_t n_s, int32_t *out_r, int32_t *out_s,
                              uint64_t capacity, uint64_t *count, void *workspace,
                              uint64_t workspace_bytes, void *stream, tj_stats_t *stats);

/*
 * Serving loop: requests of uneven sizes, admitted against a device-memory
 * budget and run concurrently.
 *
 * The paper measures the tensor path by its tail latency under a memory
 * budget (P50/P99 at a given work_mem, Sec. V-VI). A server turns that into a
 * running service: requests (sorts and joins over caller-resident device
 * columns) arrive at any time; each is admitted, in arrival order, as soon as
 * one of `slots` worker slots is idle and the arena holds its workspace and
 * outputs; admitted requests run at once on their slot's own HIP stream, so
 * small requests overlap on the GPU instead of waiting for one another.
 *
 * Memory: the caller hands the server one device arena (arena_bytes, 256-byte
 * aligned): the budget for the requests' workspaces (the work_mem of the
 * paper), which the server sub-allocates; it allocates no device memory
 * itself. Inputs and outputs are the caller's, as in the plain calls. A
 * request is admitted with the workspace it needs to finish; a join
 * materialisation is one call (TJ_E_CAPACITY with the count when its pairs
 * exceed `capacity`). Admitted work never waits for memory and releases its
 * workspace when it ends, so the queue always drains. Each request takes the
 * full workspace of its shape when that fits the arena, else the smallest one
 * (key ranges); a request whose smallest workspace exceeds the arena
 * completes at once with TJ_E_WORKSPACE.
 *
 * Fusion (continuous batching of small requests): when the head of the queue
 * is a small sort or join materialisation (rows, both sides of a join, at most
 * the server's fuse_max_rows; radix partitioner), the worker that admits it
 * also takes the queued requests of the same op and key type that are small
 * (up to fuse_max_requests and 16 * fuse_max_rows rows together, from the
 * next 256 queued) and serves them with ONE composite-key call whose leading
 * key column is the request's index in the batch. Each request's rows stay
 * together in its own stable order, and its pairs form one contiguous stretch
 * in its own canonical order, so every result equals the request run alone;
 * one set of kernel launches replaces one per request. The fused call takes
 * one arena block (combined columns, outputs and workspace); a join batch in
 * which some request's pairs exceed its own capacity is served one request at
 * a time in that block. result->fused reports the batch size.
 *
 * All functions are thread-safe. Inputs must stay valid and unchanged, and
 * outputs untouched, until the request completes.
 */
typedef struct tj_server tj_server_t;
typedef struct {
    int op;                      /* TJ_OP_SORT, TJ_OP_JOIN_COUNT or TJ_OP_JOIN_MATERIALIZE */
    int key_type;
    const void *r_keys;          /* sort: the relation to sort */
    const int32_t *r_rids;       /* sort and materialise */
    uint64_t n_r;
    const void *s_keys;          /* joins */
    const int32_t *s_rids;       /* materialise */
    uint64_t n_s;
    void *out0;                  /* sort: keys_out[n_r]; materialise: out_r[capacity] (device) */
    int32_t *out1;               /* sort: rids_out[n_r]; materialise: out_s[capacity] */
    uint64_t capacity;           /* materialise: pairs out0/out1 hold */
    uint32_t partitioner;        /* a tj_partitioner value (tj_options_t defaults otherwise) */
    uint32_t pad;
} tj_request_t;
typedef struct {
    int status;                  /* TJ_OK or the call's error */
    int op;
    uint64_t count;              /* sort: rows; joins: |R join S| (also on TJ_E_CAPACITY) */
    double queue_ms;             /* submission to admission */
    double run_ms;               /* time on a slot */
    double total_ms;             /* submission to completion */
    uint32_t learned;            /* the call used the learned first pass */
    uint32_t key_ranges;         /* tj_stats_t.key_ranges of the call */
    uint32_t fused;              /* requests served by the same call (1: alone) */
    uint32_t windows;            /* tj_stats_t.windows of the call */
} tj_result_t;
/* Starts `slots` (1..64) worker threads with one HIP stream each (default
 * priority) on the current device. Errors: TJ_E_ARG, TJ_E_WORKSPACE
 * (arena misaligned or smaller than 64 KiB), TJ_E_HIP. */
int tj_server_create(void *arena, uint64_t arena_bytes, int slots, tj_server_t **server);
/* Queues a copy of *req and returns its ticket. Argument errors of the request
 * (unknown op, key type or partitioner, NULL inputs or outputs, rows >= 2^31)
 * are returned here and queue nothing; so are outputs that overlap an input
 * or the arena (TJ_E_ALIAS). */
int tj_server_submit(tj_server_t *server, const tj_request_t *req, uint64_t *ticket);
/* Blocks until the request completes, copies its result and forgets the
 * ticket. Returns TJ_OK (the request's own status is result->status) or
 * TJ_E_ARG (unknown ticket, or a ticket another thread is already waiting for). */
int tj_server_wait(tj_server_t *server, uint64_t ticket, tj_result_t *result);
/* Fusion settings: requests of at most fuse_max_rows rows are fused, at most
 * fuse_max_requests (2 .. 256) per call; fuse_max_rows = 0 or
 * fuse_max_requests < 2 turns fusion off. Defaults: 65536 rows, 32 requests.
 * Applies to requests admitted after the call. Errors: TJ_E_ARG. */
int tj_server_configure(tj_server_t *server, uint64_t fuse_max_rows, uint32_t fuse_max_requests);
/* Arena bytes reserved now and at most so far (workspaces of running requests). */
int tj_server_memory(tj_server_t *server, uint64_t *in_use, uint64_t *peak);
/* Finishes every queued request, stops the workers and frees the server
 * (not the arena). Results not yet waited for are dropped. */
int tj_server_destroy(tj_server_t *server);

/*
 * Execution-time path selection (Sec. III.C; evaluated in Sec. V.D).
 *
 * The paper keeps the optimiser's plan and decides only at execution time
 * whether a large join or sort runs on the tensor path or on the existing
 * CPU (linear) path, from indicators that are cheap to observe then: the
 * input scale, the cardinality of the join attribute and the expected size
 * of the intermediate result. tj_select_path observes them on the device
 * columns and returns the decision; it runs neither path. The linear path is
 * the caller's own (a DBMS's hash join or sort), so this library contains no
 * CPU execution path.
 *
 * Indicators:
 *   scale:  n_r + n_s rows (sort: n_r).
 *   distinct_r, distinct_s, distinct_union: HyperLogLog estimates (Flajolet
 *     et al. 2007) of the distinct keys of R, of S and of R union S, from
 *     2^14 registers per relation (standard error about 0.8%). The hash of a
 *     key k (int32 keys sign-extended) is the first output of a SplitMix64
 *     generator (Steele, Lea, Flood 2014) seeded with k; register h >> 50
 *     keeps the largest rank (leading-one position, from 1) of the low 50
 *     bits, 51 when they are zero. With C[r] registers of rank r, Z = sum
 *     C[r] 2^(51 - r) as an exact integer, E = alpha_m m^2 2^51 / double(Z),
 *     alpha_m = 0.7213 / (1 + 1.079 / m); when E <= 2.5 m and C[0] > 0 the
 *     linear-counting estimate m ln(m / C[0]) replaces it.
 *   distinct_common: max(0, min(distinct_r, distinct_s, distinct_r +
 *     distinct_s - distinct_union)), the join keys present on both sides.
 *   est_output: expected |R join S| when the rows of each relation are
 *     spread evenly over its distinct keys: distinct_common * (n_r /
 *     distinct_r) * (n_s / distinct_s) (0 for an empty side; sort: 0). It
 *     underestimates skewed joins, whose heavy keys carry more than the
 *     average rows.
 * Decision: TJ_PATH_TENSOR when scale >= min_rows (reason TJ_SEL_SCALE) or,
 * for a join, est_output >= min_output (TJ_SEL_OUTPUT); otherwise
 * TJ_PATH_LINEAR. Options (may be NULL): a zero field takes its default,
 * TJ_SELECT_DEFAULT_MIN_ROWS and TJ_SELECT_DEFAULT_MIN_OUTPUT. The paper
 * leaves the thresholds open; the defaults come from a measured crossover on
 * one MI355X against a single-core CPU hash join and std::sort (built -O3
 * -march=native, inputs in host memory): over FK joins of 2^8 ... 2^22 rows per
 * side, the tensor path's join (device inputs, wall time of the call) is
 * faster from about 1,300 rows per side (scale 2,600, about 1,050 output
 * pairs) and its sort from about 1,760 rows, below which its fixed cost of
 * roughly 0.06-0.25 ms per call dominates.
 *
 *   op: TJ_OP_SORT (s_keys ignored, n_s must be 0) or a join op;
 *   r_keys[n_r], s_keys[n_s]: device key columns of key_type;
 *   registers: NULL, or device memory of 3 * TJ_SELECT_REGISTERS bytes that
 *     receives the R, S and union registers;
 *   workspace: tj_select_workspace_query bytes, 256-byte aligned;
 *   out (host): the indicators and the decision.
 * Synchronous: returns after the result is on the host. Errors: TJ_E_ARG
 * (NULL pointers, bad op or key type, sort with n_s != 0), TJ_E_TOO_LARGE,
 * TJ_E_WORKSPACE, TJ_E_ALIAS (registers overlapping an input or the
 * workspace, or the workspace overlapping an input), TJ_E_HIP.
 */
#define TJ_SELECT_REGISTERS 16384
#define TJ_SELECT_DEFAULT_MIN_ROWS (1ull << 11)
#define TJ_SELECT_DEFAULT_MIN_OUTPUT (1ull << 10)
enum tj_path { TJ_PATH_LINEAR = 0, TJ_PATH_TENSOR = 1 };
enum tj_select_reason { TJ_SEL_SCALE = 1, TJ_SEL_OUTPUT = 2 };
typedef struct {
    uint64_t min_rows;   /* scale at or above which the tensor path is taken */
    uint64_t min_output; /* join: expected output at or above which it is taken */
} tj_select_options_t;
typedef struct {
    uint64_t n_r, n_s;
    double distinct_r, distinct_s, distinct_union, distinct_common;
    double est_output;
    int32_t path;     /* enum tj_path */
    uint32_t reasons; /* TJ_SEL_* bits that chose the tensor path */
} tj_selection_t;
int tj_select_workspace_query(uint64_t n_r, uint64_t n_s, uint64_t *bytes);
int tj_select_path(int op, int key_type, const void *r_keys, uint64_t n_r, const void *s_keys, uint64_t n_s,
                   const tj_select_options_t *options, tj_selection_t *out, uint8_t *registers,
                   void *workspace, uint64_t workspace_bytes, void *stream);

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
 * tj_debug_stream_copy: copies `bytes` (a multiple of 16) from src to dst,
 *   both device pointers aligned to 16 bytes and not overlapping, with a plain
 *   16-byte-per-lane streaming kernel, asynchronously on `stream`. It gives
 *   the bandwidth a kernel that reads and writes each byte once reaches on
 *   the device, the practical ceiling the partition and leaf kernels are
 *   compared with. TJ_E_ARG for a size or alignment it does not take,
 *   TJ_E_ALIAS for overlapping buffers, TJ_E_HIP for a failed launch.
 */
#define TJ_DEBUG_FORCE_REORDER 1u
#define TJ_DEBUG_FAIL_HOST_ALLOC 2u
/*
 * tj_debug_set_flags: process-wide self-test switch for every later call.
 *   TJ_DEBUG_FORCE_REORDER: each partition tile and each join block also runs
 *   the ballot-ranked path that replaces an atomic-ranked order found out of
 *   input order; results must not change, only time. 0 turns it off.
 *   TJ_DEBUG_FAIL_HOST_ALLOC: every later sort or join call (plain, _ex,
 *   and the learned-model training) fails its first host-side allocation,
 *   before any device work; the call returns TJ_E_INTERNAL. It tests that no
 *   C++ exception crosses the C ABI.
 *   Returns TJ_OK, or TJ_E_ARG for unknown bits.
 */
int tj_debug_set_flags(uint32_t flags);
int tj_debug_wave_scan(const uint32_t *in, uint32_t *out, uint64_t n, void *stream);
int tj_debug_stream_copy(const void *src, void *dst, uint64_t bytes, void *stream);
int tj_debug_partition_pass(const int64_t *keys, const int32_t *rids, uint64_t n,
                            uint64_t base, uint32_t shift, uint32_t bits, uint32_t flags,
                            int64_t *keys_out, int32_t *rids_out, uint32_t *counts_out,
                            void *workspace, uint64_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TJ_H */

// tj_internal.h - descriptors shared by the host planner and the gfx950 kernels.
//
// Rows live in three places ("buffers"): 0 = the caller's input columns,
// 1 = ping buffer A, 2 = pong buffer B. Each buffer has one key column and one
// rid column per side (side 0 = R or the relation being sorted, side 1 = S).
// A partition pass reads the rows of a segment from one buffer and writes them,
// grouped by digit, to the same index range of the other buffer, so a segment's
// rows always occupy the same index range whichever buffer holds them.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "tj.h"

namespace tj {

constexpr int MAX_DIGIT_BITS = 9;             // widest partition digit
constexpr int NB = 1 << MAX_DIGIT_BITS;       // digit bins per group (table stride)
constexpr int PART_THREADS = 1024;            // histogram block
constexpr int PART_TILE = 9216;               // rows per scatter tile (chunks are multiples)
constexpr int CBLOCK = 32;                    // chunks per first-level scan block

enum Buf : uint32_t { BUF_IN = 0, BUF_A = 1, BUF_B = 2 };

// One contiguous run of a group's rows; one histogram and one scatter block.
struct ChunkDesc {
    uint64_t start;   // first row of the chunk in the source array
    uint32_t len;     // rows
    uint32_t group;   // owning group
    uint32_t cblock;  // owning scan block
    uint32_t pad;
};

// A run of consecutive chunks of one group, reduced by one first-level scan block.
struct CBlockDesc {
    uint32_t group;
    uint32_t chunk0;
    uint32_t nchunks;
    uint32_t pad;
};

// One side of one segment being partitioned in a pass.
// GroupDesc::flags: the scatter writes every tile twice, the second time
// ranked by ballot match (exercises the path taken when the ranks of a tile
// come out of input order; used by the self-test hook only).
constexpr uint32_t GROUP_FORCE_REORDER = 1u;
// GroupDesc::flags: in a launch that narrows keys to 4 bytes, this group keeps
// its 8-byte keys (its children still span more than 2^32 ordinals).
constexpr uint32_t GROUP_WIDE = 2u;
// GroupDesc::flags: the group's digit range comes from a sampled probe; the
// histogram flags any row outside [base, base + (nbins << shift)).
constexpr uint32_t GROUP_CHECK_RANGE = 4u;
// The group splits three ways around one key instead of by a radix digit:
// digit 0, 1, 2 for ord < base, ord == base, ord > base (bits = 2, shift 0;
// keys keep their width).
constexpr uint32_t GROUP_PIVOT = 8u;

struct GroupDesc {
    uint64_t start;      // first row scanned in the source array
    uint64_t len;        // rows scanned
    uint64_t dst_start;  // first row of the group in the destination array
    uint64_t base;       // ordinal subtracted before the shift
    uint64_t flo, fhi;   // only rows with flo <= ord <= fhi take part
    uint32_t shift;      // digit = (ord - base) >> shift (GROUP_PIVOT: the side of base)
    uint32_t bits;       // digit width, nbins = 1 << bits
    uint32_t side;       // column set: 0 = R / sorted relation, 1 = S
    uint32_t src, dst;   // buffers
    uint32_t chunk0, nchunks;
    uint32_t cblock0, ncblocks;
    uint32_t child0;     // first entry of this group's children in the packed child tables
    uint32_t flags;      // GROUP_* bits
    uint32_t pad;
    // Key arrays are addressed at (row + koff). Keys narrowed to 4 bytes are
    // kept inside the byte footprint of the 8-byte keys of the bucket that
    // narrowed them: koff = that bucket's first row (see the planner).
    uint64_t src_koff, dst_koff;
};

// One per-bucket LDS block: a run of adjacent final buckets of one level.
struct LeafDesc {
    uint64_t r0, s0;     // first row of each side in the buffer
    uint64_t kr0, ks0;   // index of the first row's key in each side's key array
    uint64_t base;       // ordinal subtracted before sorting inside the block
    uint64_t out;        // sort: output index of the first row; join: range base + pairs of
                         // the single-key units before this block in key order
    uint32_t rn, sn;     // rows per side (sn = 0 for the sort)
    uint16_t bits;       // significant bits of (ord - base) over the block's rows
    uint16_t kb;         // key bytes of the rows in the buffer (host bookkeeping)
    uint16_t buf;        // buffer holding the rows
    uint16_t flags;      // LEAF_* bits
};

// LeafDesc::flags: the join block sorts its rows a second time with ballot
// ranking (exercises the path taken when the atomic-ranked order fails its
// check; set by the self-test hook only).
constexpr uint16_t LEAF_FORCE_REORDER = 1u;

// A bucket whose rows all hold one key: join output is the full cross product.
// Its first pair goes to out + (pair prefix of the per-bucket joins before it).
struct CrossDesc {
    uint64_t r0, s0;     // first row of each side in the buffer
    uint64_t a, b;       // rows of R and of S
    uint64_t out;        // range base + pairs of earlier single-key units
    uint64_t pfx;        // first pair of this unit in the launch's flattened pair sequence
    uint32_t buf;
    uint32_t leaf_before;  // per-bucket joins before this unit in key order (status slot)
};

// A sort bucket of one key that is not yet in the output columns: plain copy.
struct CopyDesc {
    uint64_t start;      // first row in the buffer
    uint64_t len;
    uint64_t out;        // first output row
    uint64_t pfx;        // first row of this unit in the launch's flattened row sequence
    uint32_t buf, pad;
};

// A child bucket after a pass, both sides folded: rows per side and the
// smallest / largest key ordinal present (lo > hi when the bucket is empty).
struct ChildRec {
    uint32_t rn, sn;
    uint64_t lo, hi;
};

// Device-side leaf batching of one launch batch (k_batch_leaves).
struct BatchArgs {
    uint32_t nseg;        // segments of the launch (groups / nside)
    uint32_t nside;       // 2 for a join, 1 for a sort
    uint32_t narrowing;   // this pass narrowed the keys (children get relative ranges)
    uint32_t join;        // leaves need rows on both sides to be kept
    uint32_t buf;         // buffer holding the children
    uint32_t kb;          // key bytes of the children
    uint32_t flags;       // LeafDesc flags to set
    uint32_t leaf_base;   // first leaf slot of this batch
    uint32_t leaf_cap;    // leaf slots available in total
    uint32_t pad;
    uint64_t out_delta;   // sort: output row of buffer row 0
};
// Summary words written by k_batch_leaves (pass 1): [0] leaves, [1] rows,
// [2] flags, [4] children listed for the host ([3] is not touched).
constexpr uint64_t BATCH_WIDE = 2;        // a leaf spans more than 32 key bits
constexpr uint64_t BATCH_OVERFLOW = 4;    // the leaf slots ran out

// A child too large for one leaf (it needs another pass, or is a single key),
// listed by k_batch_leaves for the host planner in the top slots of the leaf
// table: the k-th listed child of a batch sits in slot leaf_cap - 1 - k.
struct BigChild {
    uint32_t seg, child;    // segment of the batch, digit
    uint32_t r_off, s_off;  // rows of the segment's sides before this child
    uint32_t rn, sn;
    uint64_t lo, hi;        // as in ChildRec
};
static_assert(sizeof(BigChild) <= sizeof(LeafDesc), "a listed child takes one leaf slot");

struct BufSet {
    const void* key[3][2];
    const int32_t* rid[3][2];
};

// Per-row bucket ids of the learned pass, one array per side, indexed like the
// rows of the pass's source buffer (written by the histogram, read by the scatter).
struct BktSet {
    uint16_t* b[2];
};

// One key to read back: its address in a buffer and its width (4 or 8 bytes).
struct KeyRef {
    const void* p;
    uint32_t kb, pad;
};

// Rows per leaf block (the block shape depends on the key word, see the kernels).
constexpr int LEAF_CAP = 8192;

// ---------------------------------------------------------------------------
// Launchers (tj_kernels.hip). key_bytes is 4 or 8. All return hipSuccess or the
// launch error.
// ---------------------------------------------------------------------------
hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st);
hipError_t launch_probe(int key_bytes, const void* a, uint64_t na, const void* b, uint64_t nb,
                        uint64_t* minmax, hipStream_t st);
// Min and max ordinal of every step-th element of a and of b (step 1: all).
// out[i] = ordinal of a[i * step], i < ceil(n / step)
hipError_t launch_gather_step(int key_bytes, const void* a, uint64_t n, uint64_t step, uint64_t* out, hipStream_t st);
// out[i] = ordinal of the key at refs[i] (one 4- or 8-byte key each).
hipError_t launch_read_ords(const KeyRef* refs, uint32_t n, uint64_t* out, hipStream_t st);
hipError_t launch_probe_step(int key_bytes, const void* a, uint64_t na, const void* b, uint64_t nb,
                             uint64_t step, uint64_t* minmax, hipStream_t st);
// range_miss: set to nonzero when a GROUP_CHECK_RANGE group has a row outside its digit range.
hipError_t launch_hist(int key_bytes, const ChunkDesc* chunks, uint32_t nchunks,
                       const GroupDesc* groups, BufSet bufs, uint32_t* hist,
                       uint64_t* gmin, uint64_t* gmax, uint32_t* range_miss, hipStream_t st);
// Histogram of the learned pass: the digit is the bucket of `model` (device
// copy), and each row's bucket is also stored in bkt.b[side][row].
hipError_t launch_learned_hist(int key_bytes, const ChunkDesc* chunks, uint32_t nchunks,
                               const GroupDesc* groups, BufSet bufs, const tj_rmi_t* model, BktSet bkt,
                               uint32_t* hist, uint64_t* gmin, uint64_t* gmax, hipStream_t st);
hipError_t launch_scan(const CBlockDesc* cblocks, uint32_t ncblocks, const GroupDesc* groups,
                       uint32_t ngroups, uint32_t* hist, uint32_t* cbsum, uint32_t* ccount,
                       uint64_t* cstart, hipStream_t st);
// out_key_bytes < key_bytes (8 -> 4) writes narrowed keys (see k_scatter).
hipError_t launch_scatter(int key_bytes, int out_key_bytes, bool rids, bool keys, const ChunkDesc* chunks,
                          uint32_t nchunks, const GroupDesc* groups, const uint32_t* hist,
                          const uint32_t* cbsum, const uint64_t* cstart, BufSet bufs, hipStream_t st);
// Scatter of the learned pass: digits are read from bkt (no narrowing).
hipError_t launch_learned_scatter(int key_bytes, bool rids, const ChunkDesc* chunks, uint32_t nchunks,
                                  const GroupDesc* groups, const uint32_t* hist, const uint32_t* cbsum,
                                  const uint64_t* cstart, BufSet bufs, BktSet bkt, hipStream_t st);
// Folds each segment's per-side child tables into ChildRec records, written at
// group.child0 / nside (groups come in side order per segment).
hipError_t launch_children(const GroupDesc* groups, uint32_t ngroups, int nside,
                           const uint32_t* ccount, const uint64_t* gmin, const uint64_t* gmax,
                           ChildRec* out, hipStream_t st);
// pass 0 counts each segment's leaves into seg_count; pass 1 writes them and
// adds to summary[0..2] (which the caller clears first).
hipError_t launch_batch_leaves(const GroupDesc* groups, const ChildRec* crec, const BatchArgs& a,
                               uint32_t* seg_count, LeafDesc* leaves, uint64_t* summary, int pass,
                               hipStream_t st);
hipError_t launch_leaf_sort(int key_bytes, bool wide, const LeafDesc* leaves, uint32_t n,
                            BufSet bufs, void* out_k, int32_t* out_r, hipStream_t st);
// Count mode adds the leaves' pair counts to *total. Materialise mode needs
// status[0] = inclusive-flagged carry-in offset, status[1..n] = 0, *ticket = 0;
// afterwards status[n] holds the inclusive pair total and *err != 0 flags an
// expired look-back.
hipError_t launch_leaf_join(int key_bytes, bool wide, bool materialize, const LeafDesc* leaves,
                            uint32_t n, BufSet bufs, uint64_t* status, uint32_t* ticket,
                            uint64_t* total, uint32_t* err, int32_t* out_r, int32_t* out_s,
                            uint64_t capacity, hipStream_t st);
hipError_t launch_cross(const CrossDesc* units, uint32_t n, uint64_t total, BufSet bufs,
                        const uint64_t* status, int32_t* out_r, int32_t* out_s, uint64_t capacity,
                        hipStream_t st);
constexpr uint64_t STATUS_INCLUSIVE = 2ull << 62;   // flag of a published inclusive prefix
constexpr uint64_t STATUS_VALUE = (1ull << 62) - 1;
hipError_t launch_copy(int key_bytes, const CopyDesc* units, uint32_t n, uint64_t total,
                       BufSet bufs, void* out_k, int32_t* out_r, hipStream_t st);
hipError_t launch_expand(int32_t* dst, const int32_t* src, uint64_t n, uint64_t b, int mode,
                         hipStream_t st);
hipError_t launch_wave_scan_test(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t st);

// Composite keys (tj_multi.hip). Rows r < n_a come from the col_a columns,
// rows n_a.. from col_b (a relation pair seen as one set of rows).
constexpr int MAX_KEY_COLS = 8;
struct PackArgs {
    const void* col_a[MAX_KEY_COLS];
    const void* col_b[MAX_KEY_COLS];
    uint64_t min[MAX_KEY_COLS];     // column minimum (ordinal), subtracted before the shift
    uint32_t shift[MAX_KEY_COLS];   // bit position of the column in the packed key; 64: no bits
    int32_t kb[MAX_KEY_COLS];       // key bytes of the column (4 or 8)
    uint64_t n_a;
    int32_t ncols;
    int32_t pad;
};
// out[i] = packed key of row perm[i] (perm NULL: row i), stored as a signed
// key of out_bytes (4 or 8) bytes that orders like the packed unsigned value.
hipError_t launch_pack(const PackArgs& a, const int32_t* perm, uint64_t n, void* out, int out_bytes, hipStream_t st);
// flag[i] = 1 if the key tuple of row perm[i] differs from that of row perm[i - 1] (flag[0] = 1).
hipError_t launch_tuple_flags(const PackArgs& a, const int32_t* perm, uint64_t n, uint32_t* flag, hipStream_t st);
hipError_t launch_gather(int elem_bytes, const void* in, const int32_t* perm, uint64_t n, void* out, hipStream_t st);
hipError_t launch_iota(int32_t* out, uint64_t n, hipStream_t st);
hipError_t launch_scatter_back(const uint32_t* src, const int32_t* perm, uint64_t n, int32_t* dst, hipStream_t st);
// Inclusive prefix sum of n uint32 values; scratch needs scan_scratch_words(n) words.
uint64_t scan_scratch_words(uint64_t n);
hipError_t launch_incl_scan(const uint32_t* in, uint64_t n, uint32_t* scratch, uint32_t* out, hipStream_t st);

// Learned partitioner (tj_rmi.hip).
// Rows floor(i n / m), i < m, of keys[n] to out[off + i]; rids[off + i] = off + i.
hipError_t launch_rmi_sample(int key_bytes, const void* keys, uint64_t n, uint32_t m, void* out,
                             int32_t* rids, uint32_t off, hipStream_t st);
// Fits *model to the sorted sample[M] with F buckets; start needs LEAVES + 1 words.
hipError_t launch_rmi_fit(int key_bytes, const void* sorted, uint32_t M, uint32_t F, uint32_t* start,
                          tj_rmi_t* model, hipStream_t st);
// out[i] = bucket of keys[i] under the device model.
hipError_t launch_rmi_eval(int key_bytes, const void* keys, uint64_t n, const tj_rmi_t* model,
                           uint16_t* out, hipStream_t st);


// plain streaming copy of `bytes` (a multiple of 16, both pointers 16-byte aligned)
hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t st);

// One request of a fused serving call (tj_fuse.hip): its inputs and outputs,
// rows per side, and where its rows sit in the combined columns.
struct FuseDesc {
    const void* r_keys;
    const int32_t* r_rids;
    const void* s_keys;
    const int32_t* s_rids;
    void* out0;            // sort: keys_out; join: out_r
    int32_t* out1;         // sort: rids_out; join: out_s
    uint64_t n_r, n_s;
    uint64_t off_r, off_s; // first row in the combined columns
    uint64_t capacity;     // join: pairs out0/out1 hold
};
// gather: rows of every request into the combined columns (item index, keys,
// and the request's row ids, or with positions != 0 the combined position)
hipError_t launch_fuse_gather(int key_bytes, const FuseDesc* desc, uint32_t nreq, uint64_t max_rows, int side,
                              int positions, int32_t* item, void* keys, int32_t* rids, hipStream_t st);
hipError_t launch_fuse_scatter_sort(int key_bytes, const FuseDesc* desc, uint32_t nreq, uint64_t max_rows,
                                    const void* keys, const int32_t* rids, hipStream_t st);
hipError_t launch_fuse_bounds(const int32_t* pr, const int32_t* item_r, uint64_t count, uint32_t nreq,
                              uint64_t* bounds, hipStream_t st);
hipError_t launch_fuse_scatter_pairs(const FuseDesc* desc, uint32_t nreq, const uint64_t* bounds, const int32_t* pr,
                                     const int32_t* ps, uint64_t count, hipStream_t st);

}  // namespace tj

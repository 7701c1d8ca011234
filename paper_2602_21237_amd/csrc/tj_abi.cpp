// tj_abi.cpp - host planner and the C-ABI entry points (include/tj.h).
//
// The planner drives the MSD radix plan of the tensor path:
//   probe   min / max ordinal of the keys (the "axis" extent, Sec. III.B);
//   passes  histogram + scan + stable scatter, splitting every bucket that is
//           larger than one LDS block by the next digit of its own key range
//           (the step-by-step relocation of Sec. IV.B, the alignment of both
//           relations on the join axis of Sec. IV.A);
//   leaves  runs of adjacent small buckets, each sorted (sort) or sorted and
//           matched (join) inside one LDS block;
//   singles buckets holding one key value: copied (sort) or expanded as a
//           cross product (join).
// Only the join pairs are materialised, and only at the end (Sec. III.A).
// Between passes the planner reads back the child-bucket table (sizes and key
// ranges) to size the next launch; no row data crosses to the host.
//
// Workspace budget (the work_mem analogue, Sec. VI Eq. 1): when the caller's
// workspace cannot hold the ping-pong buffers for all rows, the key domain is
// cut into ranges from a coarse key histogram, each range small enough for the
// workspace, and each range is processed on its own; its first pass scans the
// whole input and keeps only the range's rows. The extra input scans are the
// GPU counterpart of the spill term alpha(N, M).
#include "tj_internal.h"
#include "../../include/tj.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

namespace tj {
namespace {

constexpr uint64_t ALIGN = 256;
constexpr int TABLE_TIERS = 9;
constexpr uint64_t TARGET_CHUNKS = 2048;  // blocks per partition pass
#ifndef TJ_PASS_DIGIT_BITS
#define TJ_PASS_DIGIT_BITS MAX_DIGIT_BITS
#endif
// widest digit a partition pass uses (at most MAX_DIGIT_BITS)
constexpr int PASS_DIGIT_BITS = TJ_PASS_DIGIT_BITS;
constexpr size_t DEVICE_BATCH_MIN_SEGS = 16;  // segments of a pass before leaves are batched on the device
// learned partitioner defaults (tj_options_t)
constexpr uint32_t LEARNED_BUCKETS = 512;        // buckets of the learned pass: one full-width digit
constexpr uint32_t DEFAULT_PERMILLE = 10;        // 1% sample per relation
constexpr uint64_t DEFAULT_LEARNED_MIN_ROWS = 1ull << 22;
constexpr uint64_t AUTO_BULK_DEN = 2;            // auto: learned when one bucket holds over 1/2 of the rows
constexpr int TJ_SWITCH_LEARNED = 100;           // internal: the auto partitioner hands over
constexpr int TJ_RANGE_MISS = 101;               // internal: a row fell outside the sampled range
constexpr uint64_t SAMPLED_PROBE_MIN_ROWS = 1ull << 22;  // rows from which the range is sampled
constexpr uint64_t SAMPLED_PROBE_STEP = 4096;            // every 4096th key
static_assert((LEARNED_BUCKETS & (LEARNED_BUCKETS - 1)) == 0 && LEARNED_BUCKETS <= (uint32_t)NB,
              "learned buckets must be one digit of the scatter");

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

inline uint32_t nbits64(uint64_t x) { return x ? 64u - (uint32_t)__builtin_clzll(x) : 0u; }

// Table capacities of one tier. A pass whose groups, chunks, scan blocks or
// child entries exceed them runs as several launch batches.
struct Caps {
    uint32_t groups, chunks, cblocks, children, leaves, units;
};

Caps tier_caps(int t)
{
    Caps c;
    if (t == 0) {
        // the smallest tier (about 270 KB), for budgets of about a megabyte:
        // a full-width digit of one join segment still fits one launch
        c.groups = 32;
        c.chunks = 64;
        c.cblocks = 32;
        c.children = 2 * NB;
        c.leaves = 256;
        c.units = 32;
        return c;
    }
    c.groups = 64u << (t - 1);
    c.chunks = 64u << (t - 1);
    c.cblocks = 64u << (t - 1);
    c.children = 4096u << (t - 1);
    c.leaves = 1024u << (t - 1);
    c.units = 64u << (t - 1);
    return c;
}

uint64_t table_bytes(const Caps& c)
{
    uint64_t b = 0;
    b += align_up(256, ALIGN);                                        // probe + scalars
    b += align_up((uint64_t)c.groups * sizeof(GroupDesc), ALIGN);
    b += align_up((uint64_t)c.chunks * sizeof(ChunkDesc), ALIGN);
    b += align_up((uint64_t)c.cblocks * sizeof(CBlockDesc), ALIGN);
    b += align_up((uint64_t)c.chunks * NB * 4, ALIGN);               // hist
    b += align_up((uint64_t)c.cblocks * NB * 4, ALIGN);              // cbsum
    const uint64_t children = c.children;
    b += align_up(children * 4, ALIGN);                               // ccount
    b += 3 * align_up(children * 8, ALIGN);                           // cstart, gmin, gmax
    b += align_up((uint64_t)c.leaves * sizeof(LeafDesc), ALIGN);
    b += align_up(((uint64_t)c.leaves + 1) * 8, ALIGN);              // look-back status
    b += align_up(children * sizeof(ChildRec), ALIGN);                // folded child records
    b += align_up((uint64_t)c.groups * 4, ALIGN);                     // leaves per segment
    const uint64_t ub = sizeof(CrossDesc) > sizeof(CopyDesc) ? sizeof(CrossDesc) : sizeof(CopyDesc);
    b += align_up((uint64_t)c.units * ub, ALIGN);
    return b;
}

// Pinned host staging, one grow-only buffer per host thread and direction.
// It is never freed (the process exit reclaims it), so no HIP call runs from a
// thread-exit destructor.
struct PinnedBuf {
    void* p = nullptr;
    size_t cap = 0;
    void* get(size_t n)
    {
        if (n <= cap) return p;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        size_t want = 1 << 20;
        while (want < n) want *= 2;
        if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) return nullptr;
        cap = want;
        return p;
    }
};
thread_local PinnedBuf* t_down = nullptr;
thread_local PinnedBuf* t_up[2] = {nullptr, nullptr};

// Set while a call runs without allocating (tj_sort_static): read-backs then
// land in grow-only pageable host memory instead of pinned staging, and the
// call records no timing events.
thread_local bool t_noalloc = false;
thread_local std::vector<char>* t_pageable = nullptr;  // never freed, like the pinned staging

void* pinned_down(size_t n)
{
    if (t_noalloc) {
        if (!t_pageable) t_pageable = new std::vector<char>();
        if (t_pageable->size() < n) t_pageable->resize(std::max<size_t>(n, 1 << 16));
        return t_pageable->data();
    }
    if (!t_down) t_down = new PinnedBuf();
    return t_down->get(n);
}

void* pinned_up(size_t n, int slot)
{
    if (t_noalloc) return nullptr;  // uploads then go from the caller's pageable memory
    if (!t_up[slot]) t_up[slot] = new PinnedBuf();
    return t_up[slot]->get(n);
}

// Host-to-device copy of a planner table on `st`. Large tables go through a
// pinned staging buffer (a pageable source is copied in small synchronous
// pieces), one per slot (0: leaves, 1: cross or copy units); the caller
// synchronises `st` before it writes the next upload of the same slot.
hipError_t upload(void* dst, const void* src, size_t bytes, hipStream_t st, int slot)
{
    void* pin = bytes >= (256u << 10) ? pinned_up(bytes, slot) : nullptr;
    if (!pin) return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    std::memcpy(pin, src, bytes);
    return hipMemcpyAsync(dst, pin, bytes, hipMemcpyHostToDevice, st);
}

// Bytes of one row in the ping-pong buffers.
inline uint64_t row_bytes(int kb, bool rids) { return (uint64_t)kb + (rids ? 4u : 0u); }

struct Shape {
    int op, kb;
    bool join, mat, rids;
    uint64_t n_r, n_s;
};

// Bytes of the ping-pong buffers of the unlimited plan: the sort keeps one
// buffer in the workspace (its other buffer is the caller's output), the join
// two per side.
uint64_t buffer_data_bytes(const Shape& s)
{
    const int nbuf = s.join ? 2 : 1;
    uint64_t b = 0;
    for (int buf = 0; buf < nbuf; buf++)
        for (uint64_t n : {s.n_r, s.n_s}) {
            if (n == 0) continue;
            b += align_up(n * (uint64_t)s.kb, ALIGN);
            if (s.rids) b += align_up(n * 4, ALIGN);
        }
    return b;
}

// Smallest data region: ping and pong buffers of 2048 rows per side (a key
// range only has to hold its own rows; smaller budgets just mean more ranges),
// plus alignment slack.
uint64_t min_data_bytes(const Shape& s)
{
    const uint64_t per = align_up(2048ull * row_bytes(s.kb, s.rids), ALIGN) * 2 + 16 * ALIGN;
    return s.join ? 2 * per : per;
}

const uint64_t kMaxRows = (1ull << 31) - 1;

// Digit of a pass over a segment of `rows` rows whose ordinals span `span`:
// enough digits that a child averages LEAF_CAP / 2 rows (at least 2, at most a
// full digit), at the largest shift at which (span >> shift) + 1 digits still
// reach that many, so a span that is not a power of two still puts them to
// use. With `few` (a level of at most FEW_SEGS segments) a segment of at most
// SMALL_SEG_ROWS rows (mostly a bucket crowded by a few frequent keys) takes
// a full digit: such a level costs about its launches and read-back whatever
// the width, and the wider digit separates the frequent keys from their
// neighbours in fewer levels. (A level of many segments keeps the narrower
// digit: the children's bookkeeping grows with the width.) A span of 0
// (filtered roots of a single-key range, which still need a compaction pass)
// gets one bit.
constexpr uint64_t SMALL_SEG_ROWS = 16ull * LEAF_CAP;
constexpr size_t FEW_SEGS = 64;
// A child bucket is crowded (Seg::skew) when it holds more than SKEW_FACTOR
// times the rows its parent's digit gave each bucket on average; at most
// MAX_PIVOT_SEGS crowded buckets of a level are sampled for a pivot key.
constexpr uint64_t SKEW_FACTOR = 2;
constexpr size_t MAX_PIVOT_SEGS = 4096;
inline void plan_digit(uint64_t span, uint64_t rows, bool few, uint32_t& shift, uint32_t& bits)
{
    const uint64_t want =
        few && rows <= SMALL_SEG_ROWS
            ? 1ull << PASS_DIGIT_BITS
            : std::min<uint64_t>(std::max<uint64_t>((rows + LEAF_CAP / 2 - 1) / (LEAF_CAP / 2), 2),
                                 1ull << PASS_DIGIT_BITS);
    shift = 0;
    for (uint32_t sh = nbits64(span); sh-- > 0;)
        if ((span >> sh) + 1 >= want) {
            shift = sh;
            break;
        }
    while ((span >> shift) >= (1ull << PASS_DIGIT_BITS)) shift++;
    bits = std::max<uint32_t>(1, nbits64(span >> shift));
}

// Sample rows of a relation of n rows: max(min(n, 2048), n * permille / 1000).
inline uint64_t rmi_sample_rows(uint64_t n, uint32_t permille)
{
    const uint64_t a = std::min<uint64_t>(n, 2048), b = n * permille / 1000;
    return std::max(a, b);
}

// Training scratch of the learned partitioner for M sample rows: the sample,
// its sorted copy (keys and rids), the leaf run starts, and a workspace for
// the sample's sort (`full`: the sort's unlimited workspace, else its minimum).
uint64_t rmi_scratch_bytes(int kb, uint64_t M, bool full)
{
    const Shape ss{TJ_OP_SORT, kb, false, false, true, M, 0};
    const uint64_t sort_ws = full ? table_bytes(tier_caps(TABLE_TIERS - 1)) + buffer_data_bytes(ss)
                                  : table_bytes(tier_caps(0)) + min_data_bytes(ss);
    return 2 * align_up(M * (uint64_t)kb, ALIGN) + 2 * align_up(M * 4, ALIGN) +
           align_up((TJ_RMI_LEAVES + 1) * 4, ALIGN) + sort_ws;
}

// Buffer B during a learned call: [model][per-row buckets of R][of S] for the
// learned pass, the training scratch after the model before it.
uint64_t rmi_model_bytes() { return align_up(sizeof(tj_rmi_t), ALIGN); }

// Data bytes of the unlimited plan: the ping-pong buffers, and at least room
// in buffer B (free until the second pass) to train the learned partitioner
// at its default sample rate.
uint64_t full_data_bytes(const Shape& s)
{
    const uint64_t buffers = buffer_data_bytes(s);
    uint64_t b_off = 0;  // buffer B follows buffer A (join); the sort's B starts the region
    if (s.join) {
        const Shape a{s.op, s.kb, false, s.mat, s.rids, s.n_r, s.n_s};
        b_off = buffer_data_bytes(a);
    }
    const uint64_t M = rmi_sample_rows(s.n_r, 10) + (s.join ? rmi_sample_rows(s.n_s, 10) : 0);
    const uint64_t n = s.n_r + (s.join ? s.n_s : 0);
    const uint64_t need = rmi_model_bytes() + std::max(rmi_scratch_bytes(s.kb, M, false),
                                                       align_up(s.n_r * 2, ALIGN) + align_up(s.n_s * 2, ALIGN));
    (void)n;
    return std::max(buffers, b_off + need);
}

// ---------------------------------------------------------------------------
// The executor of one call.
// ---------------------------------------------------------------------------
struct Seg {
    uint64_t r0, rn, s0, sn;  // row ranges (side 0, side 1)
    uint64_t lo, hi;          // ordinal range present (lo > hi: no rows)
    uint32_t buf;
    uint32_t kb = 0;          // key bytes of the rows in `buf`
    // Narrowed keys (kb 4 of an int64 input) hold ord - win; win is the
    // original ordinal of their 2^32-aligned window. ~0: keys are not narrowed.
    uint64_t win = ~0ull;
    // Row i's key sits at index i + koff of its side's key array. Narrowed
    // keys use koff = first row of the bucket that narrowed them, which keeps
    // them (4 bytes at index i + koff) inside that bucket's 8-byte footprint,
    // away from the 8-byte keys of other buckets in the same buffer.
    uint64_t koff_r = 0, koff_s = 0;
    // Under a binding budget, rows taken through a packed workspace window
    // (buffer B): row in B minus row in buffer A of the same data, for side 0
    // (the sort's rows, R) and side 1 (S); 0 everywhere else.
    int64_t wdisp = 0, wdisp_s = 0;
    // Far more rows than its radix digit gave each bucket of its parent on
    // average: likely crowded by one frequent key (see Exec::pick_pivots).
    bool skew = false;
};

struct Unit {                 // a final piece of join output, ordered by key
    uint64_t lo;
    int kind;                 // 0 leaf, 1 cross
    uint32_t index;           // into leaves / crosses
    uint64_t count;
};

#define TJ_CK(expr)                                   \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return TJ_E_HIP;        \
    } while (0)

#define TJ_RET(expr)                                  \
    do {                                              \
        int r_ = (expr);                              \
        if (r_ != TJ_OK) return r_;                   \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel timing registry (tj_timing / tj_timing_read).
// ---------------------------------------------------------------------------
enum Fam { F_PROBE, F_HIST, F_SCAN, F_SCATTER, F_LEAF_SORT, F_LEAF_COUNT, F_LEAF_MAT, F_CROSS, F_COPY,
           F_EXPAND, F_HOST_CLASSIFY, F_HOST_LEAVES, F_RMI_TRAIN, F_LHIST, F_LSCATTER, NFAM };
const char* const kFamName[NFAM] = {"probe", "histogram", "scan", "scatter", "leaf_sort",
                                    "leaf_join_count", "leaf_join_mat", "cross", "copy", "expand",
                                    "host_classify", "host_leaves", "rmi_train", "learned_hist",
                                    "learned_scatter"};

struct Timing {
    std::mutex mu;
    bool on = false;
    uint64_t launches[NFAM] = {};
    uint64_t bytes[NFAM] = {};
    double ms[NFAM] = {};
};
Timing& timing()
{
    static Timing t;
    return t;
}

// Set while a call runs the plain sort on its own sample (training of the
// learned model): that inner call's launches are timed as part of rmi_train.
thread_local int t_nested = 0;

// Process-wide self-test flags (tj_debug_set_flags).
std::atomic<uint32_t> g_debug_flags{0};

// Stable sort of (position, index) pairs by position, `top` the largest
// position: LSD radix, 11 bits a pass (planner tables hold 10^5 entries).
void radix_order(std::vector<std::pair<uint64_t, uint32_t>>& a, std::vector<std::pair<uint64_t, uint32_t>>& t,
                 uint64_t top)
{
    constexpr int D = 11;
    uint32_t cnt[1u << D];
    t.resize(a.size());
    for (int sh = 0; sh < 64 && (top >> sh); sh += D) {
        std::fill(cnt, cnt + (1u << D), 0u);
        for (const auto& p : a) cnt[(p.first >> sh) & ((1u << D) - 1)]++;
        uint32_t sum = 0;
        for (uint32_t& c : cnt) {
            const uint32_t k = c;
            c = sum;
            sum += k;
        }
        for (const auto& p : a) t[cnt[(p.first >> sh) & ((1u << D) - 1)]++] = p;
        a.swap(t);
    }
}

// Host-side lists of one call (see Exec::hv).
struct HostVecs {
    std::vector<LeafDesc> leaves, batch_leaves;
    std::vector<std::pair<uint64_t, uint32_t>> order, order_tmp;
    std::vector<BigChild> big;
    std::vector<CrossDesc> crosses, batch_crosses;
    std::vector<CopyDesc> copies;
    bool busy = false;
    void clear()
    {
        leaves.clear();
        batch_leaves.clear();
        crosses.clear();
        batch_crosses.clear();
        copies.clear();
    }
};
thread_local HostVecs* t_host_vecs = nullptr;  // never freed, like the pinned staging

// The thread's lists, or (if a call on this thread already holds them) a
// private set owned through `owned`.
HostVecs& borrow_host_vecs(HostVecs*& owned)
{
    // self-test: a host allocation failure at the start of a call, before any device work
    if (g_debug_flags.load() & TJ_DEBUG_FAIL_HOST_ALLOC) throw std::bad_alloc();
    if (!t_host_vecs) t_host_vecs = new HostVecs();
    if (!t_host_vecs->busy) {
        t_host_vecs->busy = true;
        t_host_vecs->clear();
        return *t_host_vecs;
    }
    owned = new HostVecs();
    return *owned;
}

// Frees the calling thread's staging buffers and host lists (see
// tj::release_thread_staging).
// Timing events are reused from a per-thread pool (creating and destroying
// two events per timed launch cost more host time than the launch itself).
// Each entry remembers the device it was created on.
thread_local std::vector<std::pair<int, hipEvent_t>>* t_events = nullptr;

hipEvent_t take_event()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    if (t_events)
        for (size_t i = t_events->size(); i-- > 0;)
            if ((*t_events)[i].first == dev) {
                const hipEvent_t e = (*t_events)[i].second;
                (*t_events)[i] = t_events->back();
                t_events->pop_back();
                return e;
            }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void give_event(hipEvent_t e)
{
    if (!e) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    if (!t_events) t_events = new std::vector<std::pair<int, hipEvent_t>>();
    t_events->push_back({dev, e});
}

void free_thread_staging()
{
    auto drop = [](PinnedBuf*& b) {
        if (!b) return;
        if (b->p) (void)hipHostFree(b->p);
        delete b;
        b = nullptr;
    };
    drop(t_down);
    drop(t_up[0]);
    drop(t_up[1]);
    delete t_pageable;
    t_pageable = nullptr;
    if (t_host_vecs && !t_host_vecs->busy) {
        delete t_host_vecs;
        t_host_vecs = nullptr;
    }
    if (t_events) {
        for (auto& pe : *t_events) (void)hipEventDestroy(pe.second);
        delete t_events;
        t_events = nullptr;
    }
}

void return_host_vecs(HostVecs& hv, HostVecs* owned)
{
    hv.clear();
    if (owned) delete owned;
    else hv.busy = false;
}

struct Pending {
    int fam;
    hipEvent_t a, b;
    uint64_t bytes;
};

struct Exec {
    Shape sh;
    hipStream_t st = nullptr;
    BufSet bufs{};
    Caps caps{};
    tj_stats_t stats{};

    // device tables
    uint64_t* d_probe = nullptr;
    GroupDesc* d_groups = nullptr;
    ChunkDesc* d_chunks = nullptr;
    CBlockDesc* d_cblocks = nullptr;
    uint32_t* d_hist = nullptr;
    uint32_t* d_cbsum = nullptr;
    uint32_t* d_ccount = nullptr;
    uint64_t* d_cstart = nullptr;
    uint64_t* d_gmin = nullptr;
    uint64_t* d_gmax = nullptr;
    LeafDesc* d_leaves = nullptr;
    uint64_t* d_status = nullptr;  // caps.leaves + 1 look-back words
    ChildRec* d_crec = nullptr;     // caps.children folded child records
    uint32_t* d_segcount = nullptr; // caps.groups leaf counts (device batching)
    // scalars in the probe block: [0..1] min/max, [2] pair total, [3] ticket (low) + error (high),
    // [4..6] device batching summary (leaves, rows, flags)
    void* d_units = nullptr;
    tj_rmi_t* d_model = nullptr;    // learned bucket function (when trained)
    BktSet bkt{};                   // per-row buckets of the learned pass
    bool learned_pass = false;      // the next partition pass is the learned one
    bool auto_probe = false;        // the next pass may hand over to the learned partitioner
    bool spec_range = false;        // the next pass's digit range comes from a sampled probe

    // data buffer capacities (rows per side) when the buffers live in the workspace
    uint64_t cap_r = 0, cap_s = 0;
    bool out_is_a = false;  // sort: buffer A is the caller's output
    uint64_t a_off = 0;     // sort: output row of buffer A's row 0
    // sort under a binding budget: leaves whose rows are already in the output
    // columns (rows counted from the columns' start), sorted in one launch at the end
    std::vector<LeafDesc> deferred;
    bool write_keys = true; // partition passes write key columns (off: rid-only compaction)
    bool device_batching = true;  // the last level's leaves may be batched on the device
    // join under a binding budget with every key range narrow enough that its
    // filtered pass narrows the keys to 4 bytes: that pass takes a full digit
    // (shift <= 32 is then certain) and the buffers hold 4-byte keys
    bool narrow_ranges = false;
    // the join's key ranges pack their buckets that need further passes into
    // buffer B, a window of win_r / win_s rows (layout_join_window)
    bool window = false;
    uint64_t win_r = 0, win_s = 0;
    // crowded buckets may split three ways around a frequent key
    bool pivots = true;

    // timing of this call's launches (when enabled)
    bool timed_on = false;
    std::vector<Pending> pending;

    template <class F>
    hipError_t timed(int fam, uint64_t bytes, F&& f)
    {
        if (!timed_on) return f();
        Pending p{fam, take_event(), take_event(), bytes};
        if (!p.a || !p.b) {
            give_event(p.a);
            give_event(p.b);
            return hipErrorUnknown;
        }
        hipError_t e = hipEventRecord(p.a, st);
        if (e == hipSuccess) e = f();
        if (e == hipSuccess) e = hipEventRecord(p.b, st);
        pending.push_back(p);
        return e;
    }

    // Accumulates the event durations of this call (stream already synchronised).
    void flush_timing()
    {
        if (pending.empty()) return;
        Timing& t = timing();
        std::lock_guard<std::mutex> g(t.mu);
        for (Pending& p : pending) {
            float ms = 0;
            // (the call has synchronised its stream; an error path may not have)
            hipError_t r = hipEventElapsedTime(&ms, p.a, p.b);
            if (r == hipErrorNotReady && hipEventSynchronize(p.b) == hipSuccess) r = hipEventElapsedTime(&ms, p.a, p.b);
            if (r == hipSuccess) {
                t.launches[p.fam]++;
                t.bytes[p.fam] += p.bytes;
                t.ms[p.fam] += ms;
            }
            give_event(p.a);
            give_event(p.b);
        }
        pending.clear();
    }

    ~Exec()
    {
        // A call that failed half way may leave copies from the thread's pinned
        // staging queued on its stream: they must not read what the next call
        // stages there.
        if (hipStreamQuery(st) == hipErrorNotReady) (void)hipStreamSynchronize(st);
        flush_timing();
        return_host_vecs(hv, hv_owned);
    }

    // Host planning time between a read-back and the next launch (families
    // host_*; launches counts timed sections, bytes stays 0).
    struct HostTimer {
        Exec* x;
        int fam;
        std::chrono::steady_clock::time_point t0;
        bool done = false;
        HostTimer(Exec* e, int f) : x(e), fam(f), t0(std::chrono::steady_clock::now()) {}
        ~HostTimer() { stop(); }
        void stop()
        {
            if (done || !x->timed_on) return;
            done = true;
            const double ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            Timing& t = timing();
            std::lock_guard<std::mutex> g(t.mu);
            t.launches[fam]++;
            t.ms[fam] += ms;
        }
    };

    // host-side results
    // Host-side lists live in per-thread storage that keeps its capacity from
    // call to call: a fresh multi-megabyte vector costs a page fault per 4 KiB
    // on every call, more than the planning itself.
    HostVecs* hv_owned = nullptr;
    HostVecs& hv = borrow_host_vecs(hv_owned);
    std::vector<LeafDesc>& leaves = hv.leaves;
    std::vector<CrossDesc>& crosses = hv.crosses;
    std::vector<CopyDesc>& copies = hv.copies;

    // ---- workspace layout -------------------------------------------------
    int carve_tables(char*& p, char* end)
    {
        auto take = [&](uint64_t bytes) -> char* {
            char* q = p;
            p += align_up(bytes, ALIGN);
            return q;
        };
        d_probe = (uint64_t*)take(256);
        d_groups = (GroupDesc*)take((uint64_t)caps.groups * sizeof(GroupDesc));
        d_chunks = (ChunkDesc*)take((uint64_t)caps.chunks * sizeof(ChunkDesc));
        d_cblocks = (CBlockDesc*)take((uint64_t)caps.cblocks * sizeof(CBlockDesc));
        d_hist = (uint32_t*)take((uint64_t)caps.chunks * NB * 4);
        d_cbsum = (uint32_t*)take((uint64_t)caps.cblocks * NB * 4);
        const uint64_t children = caps.children;
        d_ccount = (uint32_t*)take(children * 4);
        d_cstart = (uint64_t*)take(children * 8);
        d_gmin = (uint64_t*)take(children * 8);
        d_gmax = (uint64_t*)take(children * 8);
        d_leaves = (LeafDesc*)take((uint64_t)caps.leaves * sizeof(LeafDesc));
        d_status = (uint64_t*)take(((uint64_t)caps.leaves + 1) * 8);
        d_crec = (ChildRec*)take(children * sizeof(ChildRec));
        d_segcount = (uint32_t*)take((uint64_t)caps.groups * 4);
        const uint64_t ub = sizeof(CrossDesc) > sizeof(CopyDesc) ? sizeof(CrossDesc) : sizeof(CopyDesc);
        d_units = take((uint64_t)caps.units * ub);
        return p <= end ? TJ_OK : TJ_E_WORKSPACE;
    }

    // ---- one partition pass over a list of segments that live in `src` ----
    // Hands every child, in key order, to `sink` (called with a const Seg&)
    // as soon as its launch batch has been read back.
    template <class Sink>
    int run_pass(const std::vector<Seg>& segs, uint32_t src, uint32_t dst,
                 const uint64_t* filter, Sink&& sink)
    {
        stats.passes++;
        const int nside = sh.join ? 2 : 1;
        // the learned pass partitions the root segment(s) of an unfiltered range once
        const bool learned = learned_pass && !filter;
        learned_pass = false;
        const bool spec = spec_range && !filter && !learned;
        spec_range = false;
        // per segment digit choice
        struct Plan {
            uint32_t shift, bits, kb_out;
            bool pivot;
            uint64_t key;  // the pivot's ordinal
        };
        std::vector<Plan> plan(segs.size());
        // (calls that may not allocate keep their radix digits: their launches
        // stay the ones checked for an unchanged device memory footprint)
        if (pivots && !filter && !learned && !t_noalloc) TJ_RET(pick_pivots(segs, plan));
        uint64_t total_rows = 0;
        for (size_t i = 0; i < segs.size(); i++) {
            const Seg& s = segs[i];
            if (plan[i].pivot) {  // three children: below, equal to, above the pivot; keys keep their width
                plan[i].shift = 0;
                plan[i].bits = 2;
                plan[i].kb_out = s.kb;
                total_rows += s.rn + s.sn;
                continue;
            }
            plan_digit(s.hi - s.lo, s.rn + s.sn, segs.size() <= FEW_SEGS, plan[i].shift, plan[i].bits);
            if (filter && narrow_ranges) plan_digit(s.hi - s.lo, SMALL_SEG_ROWS, true, plan[i].shift, plan[i].bits);
            // join keys are narrowed to 4 bytes once every child spans at most
            // 2^32 ordinals; the sort writes its keys out and never narrows
            plan[i].kb_out = sh.join && write_keys && s.kb == 8 && plan[i].shift <= 32 ? 4u : s.kb;
            if (learned) {
                // the model's buckets are the digits; children keep their key width
                plan[i].bits = nbits64(LEARNED_BUCKETS) - 1;
                plan[i].shift = 0;
                plan[i].kb_out = s.kb;
            }
            total_rows += filter ? (uint64_t)(i == 0 ? sh.n_r + sh.n_s : 0) : s.rn + s.sn;
        }
        // Device batching pays where the children are many: one wave per
        // segment batches them (tens of microseconds for a level), while the
        // host needs about 5 ns per child. Children too large for a leaf are
        // listed for the host, which plans only those.
        if (segs.size() < DEVICE_BATCH_MIN_SEGS || learned) dev_ok = false;
        for (const Seg& sg : segs)
            if (sg.wdisp || sg.wdisp_s) dev_ok = false;  // device leaves: one buffer mapping
        uint64_t ch_rows = align_up((total_rows + TARGET_CHUNKS - 1) / TARGET_CHUNKS, PART_TILE);
        if (ch_rows < PART_TILE) ch_rows = PART_TILE;
        // make sure the largest group fits the chunk table
        for (size_t i = 0; i < segs.size(); i++) {
            const uint64_t lr = filter ? sh.n_r : segs[i].rn;
            const uint64_t ls = filter ? (sh.join ? sh.n_s : 0) : segs[i].sn;
            while ((lr + ch_rows - 1) / ch_rows + (ls + ch_rows - 1) / ch_rows > caps.chunks) ch_rows *= 2;
        }

        std::vector<GroupDesc> groups;
        std::vector<ChunkDesc> chunks;
        std::vector<CBlockDesc> cblocks;
        std::vector<size_t> gseg;  // group -> segment
        // Launches take one input key width. A level whose segments mix widths
        // (keys narrowed in some buckets only) runs its 8-byte segments first,
        // then its 4-byte ones, instead of a launch per run of equal widths;
        // children then reach the sink out of key order, which only the
        // device leaf batching relies on.
        std::vector<size_t> order(segs.size());
        for (size_t i = 0; i < segs.size(); i++) order[i] = i;
        bool kb_mixed = false;
        for (size_t i = 1; i < segs.size(); i++) kb_mixed = kb_mixed || segs[i].kb != segs[0].kb;
        if (kb_mixed) {
            std::stable_partition(order.begin(), order.end(), [&](size_t i) { return segs[i].kb == 8; });
            if (dev_ok) TJ_RET(demote_device_leaves());
        }
        size_t oi = 0;
        while (oi < segs.size()) {
            groups.clear();
            chunks.clear();
            cblocks.clear();
            gseg.clear();
            uint32_t child = 0;
            // fill one launch batch: its segments share the input key width; some
            // may narrow their keys while others keep them (GROUP_WIDE)
            const uint32_t kb_in = segs[order[oi]].kb;
            while (oi < segs.size()) {
                const size_t si = order[oi];
                const Seg& s = segs[si];
                if (s.kb != kb_in) break;
                uint64_t need_chunks = 0, need_cb = 0;
                for (int side = 0; side < nside; side++) {
                    const uint64_t len = filter ? (side ? sh.n_s : sh.n_r) : (side ? s.sn : s.rn);
                    const uint64_t nc = (len + ch_rows - 1) / ch_rows;
                    need_chunks += nc;
                    need_cb += (nc + CBLOCK - 1) / CBLOCK;
                }
                if (groups.size() + nside > caps.groups || chunks.size() + need_chunks > caps.chunks ||
                    cblocks.size() + need_cb > caps.cblocks ||
                    child + ((uint64_t)nside << plan[si].bits) > caps.children) {
                    if (groups.empty()) return TJ_E_WORKSPACE;
                    break;
                }
                for (int side = 0; side < nside; side++) {
                    GroupDesc g{};
                    const uint64_t len = filter ? (side ? sh.n_s : sh.n_r) : (side ? s.sn : s.rn);
                    g.start = filter ? 0 : (side ? s.s0 : s.r0);
                    g.len = len;
                    g.dst_start = side ? s.s0 : s.r0;  // a filtered root's rows start there too
                    if (!filter) {  // into or out of the window
                        const int64_t w = side ? s.wdisp_s : s.wdisp;
                        g.dst_start += (dst == BUF_B ? w : 0) - (src == BUF_B ? w : 0);
                    }
                    g.base = learned ? 0 : plan[si].pivot ? plan[si].key : s.lo;
                    g.flo = filter ? filter[0] : 0;
                    g.fhi = filter ? filter[1] : ~0ull;
                    g.shift = plan[si].shift;
                    g.bits = plan[si].bits;
                    g.side = (uint32_t)side;
                    g.src = src;
                    g.dst = dst;
                    g.chunk0 = (uint32_t)chunks.size();
                    g.cblock0 = (uint32_t)cblocks.size();
                    g.child0 = child;
                    child += 1u << g.bits;
                    g.flags = (g_debug_flags.load() & TJ_DEBUG_FORCE_REORDER) ? GROUP_FORCE_REORDER : 0u;
                    if (spec) g.flags |= GROUP_CHECK_RANGE;
                    if (plan[si].pivot) g.flags |= GROUP_PIVOT;
                    g.src_koff = filter ? 0 : (side ? s.koff_s : s.koff_r);
                    // narrowed keys: at their rows' index in 4-byte key buffers, else
                    // inside the 8-byte footprint of the bucket that narrowed them
                    g.dst_koff = plan[si].kb_out < kb_in ? (narrow_ranges ? 0 : g.dst_start) : g.src_koff;
                    const uint32_t gi = (uint32_t)groups.size();
                    for (uint64_t c0 = 0; c0 < len; c0 += ch_rows) {
                        ChunkDesc c{};
                        c.start = g.start + c0;
                        c.len = (uint32_t)std::min<uint64_t>(ch_rows, len - c0);
                        c.group = gi;
                        c.cblock = (uint32_t)(cblocks.size() + (chunks.size() - g.chunk0) / CBLOCK);
                        chunks.push_back(c);
                    }
                    g.nchunks = (uint32_t)chunks.size() - g.chunk0;
                    for (uint32_t c = 0; c < g.nchunks; c += CBLOCK) {
                        CBlockDesc b{};
                        b.group = gi;
                        b.chunk0 = g.chunk0 + c;
                        b.nchunks = std::min<uint32_t>(CBLOCK, g.nchunks - c);
                        cblocks.push_back(b);
                    }
                    g.ncblocks = (uint32_t)cblocks.size() - g.cblock0;
                    groups.push_back(g);
                    gseg.push_back(si);
                    stats.bytes_read += len * (uint64_t)kb_in;                                   // histogram
                    stats.bytes_read += len * (uint64_t)kb_in + (sh.rids ? len * 4 : 0);         // scatter
                }
                oi++;
            }
            const uint32_t ng = (uint32_t)groups.size(), nc = (uint32_t)chunks.size(),
                           ncb = (uint32_t)cblocks.size();
            // the launch narrows when any segment does; the others are marked wide
            uint32_t kb_out = kb_in;
            bool mixed = false;
            for (uint32_t gi = 0; gi < ng; gi++) kb_out = std::min(kb_out, plan[gseg[gi]].kb_out);
            for (uint32_t gi = 0; gi < ng; gi++)
                if (plan[gseg[gi]].kb_out != kb_out) {
                    groups[gi].flags |= GROUP_WIDE;
                    mixed = true;
                }
            {
                // the three tables go out from one pinned staging buffer (a copy
                // from pageable memory would block the host until it is done)
                const size_t gb = ng * sizeof(GroupDesc), cb = nc * sizeof(ChunkDesc),
                             bb = ncb * sizeof(CBlockDesc);
                char* pin = (char*)pinned_up(gb + cb + bb, 0);
                const char* hg = (const char*)groups.data();
                const char* hc = (const char*)chunks.data();
                const char* hb = (const char*)cblocks.data();
                if (pin) {
                    std::memcpy(pin, hg, gb);
                    std::memcpy(pin + gb, hc, cb);
                    std::memcpy(pin + gb + cb, hb, bb);
                    hg = pin;
                    hc = pin + gb;
                    hb = pin + gb + cb;
                }
                TJ_CK(hipMemcpyAsync(d_groups, hg, gb, hipMemcpyHostToDevice, st));
                TJ_CK(hipMemcpyAsync(d_chunks, hc, cb, hipMemcpyHostToDevice, st));
                TJ_CK(hipMemcpyAsync(d_cblocks, hb, bb, hipMemcpyHostToDevice, st));
            }
            TJ_CK(launch_fill_u64(d_gmin, child, ~0ull, st));
            TJ_CK(launch_fill_u64(d_gmax, child, 0ull, st));
            uint64_t scanned = 0, written = 0;  // rows read; bytes written
            for (const GroupDesc& g : groups) {
                scanned += g.len;
                const size_t sidx = gseg[&g - groups.data()];
                const Seg& s = segs[sidx];
                written += (g.side ? s.sn : s.rn) * ((write_keys ? plan[sidx].kb_out : 0) + (sh.rids ? 4 : 0));
            }
            const uint64_t rb = row_bytes((int)kb_in, sh.rids);
            if (learned) {
                // bucket ids: 2 bytes written per row by the histogram, read by the scatter
                TJ_CK(timed(F_LHIST, scanned * (kb_in + 2), [&] {
                    return launch_learned_hist((int)kb_in, d_chunks, nc, d_groups, bufs, d_model, bkt, d_hist,
                                               d_gmin, d_gmax, st);
                }));
                stats.bytes_written += scanned * 2;
                stats.bytes_read += scanned * 2;
            } else {
                uint32_t* miss = (uint32_t*)(d_probe + 7);
                if (spec) TJ_CK(launch_fill_u64(d_probe + 7, 1, 0, st));
                TJ_CK(timed(F_HIST, scanned * kb_in, [&] {
                    return launch_hist((int)kb_in, d_chunks, nc, d_groups, bufs, d_hist, d_gmin, d_gmax, miss, st);
                }));
                if (spec) {
                    // a row outside the sampled digit range: nothing moved yet, the
                    // caller probes the exact range and starts again
                    uint64_t* flag = (uint64_t*)pinned_down(sizeof(uint64_t));
                    if (!flag) return TJ_E_HIP;
                    TJ_CK(hipMemcpyAsync(flag, d_probe + 7, 8, hipMemcpyDeviceToHost, st));
                    TJ_CK(hipStreamSynchronize(st));
                    if (*flag) {
                        stats.passes--;
                        return TJ_RANGE_MISS;
                    }
                }
            }
            TJ_CK(timed(F_SCAN, 0, [&] {
                return launch_scan(d_cblocks, ncb, d_groups, ng, d_hist, d_cbsum, d_ccount, d_cstart, st);
            }));
            if (auto_probe) {
                // The radix digit's bucket sizes decide. Every next pass
                // narrows the digit to its bucket's own key range, so a few
                // dense key intervals split at the next level; but when one
                // bucket holds most of the rows, the digit has not separated
                // the bulk of the keys from a long tail, and narrowing leaves
                // it crowded again level after level: then the learned
                // partitioner takes over (nothing has been scattered yet).
                auto_probe = false;
                std::vector<uint32_t> cnt(child);
                TJ_CK(hipMemcpyAsync(cnt.data(), d_ccount, (size_t)child * 4, hipMemcpyDeviceToHost, st));
                TJ_CK(hipStreamSynchronize(st));
                uint64_t rows = 0, largest = 0;
                std::vector<uint64_t> per(child / nside, 0);
                for (uint32_t gi = 0; gi < ng; gi++)
                    for (uint32_t d = 0; d < (1u << groups[gi].bits); d++)
                        per[groups[gi - gi % nside].child0 / nside + d] += cnt[groups[gi].child0 + d];
                for (uint64_t c : per) {
                    rows += c;
                    largest = std::max(largest, c);
                }
                if (AUTO_BULK_DEN * largest > rows) {
                    stats.passes--;  // histogram only
                    return TJ_SWITCH_LEARNED;
                }
            }
            if (learned) {
                TJ_CK(timed(F_LSCATTER, scanned * (rb + 2) + written, [&] {
                    return launch_learned_scatter((int)kb_in, sh.rids, d_chunks, nc, d_groups, d_hist, d_cbsum,
                                                  d_cstart, bufs, bkt, st);
                }));
            } else {
                TJ_CK(timed(F_SCATTER, scanned * rb + written, [&] {
                    return launch_scatter((int)kb_in, (int)kb_out, sh.rids, write_keys, d_chunks, nc, d_groups, d_hist,
                                          d_cbsum, d_cstart, bufs, st);
                }));
            }
            // one compact record per child (both sides folded)
            const uint32_t nrec = child / (uint32_t)nside;
            // Child d of the segment whose first group is gi, with rows [r0, ..) and
            // [s0, ..) in the destination: a Seg for the sink. Its keys may have been
            // narrowed by this pass; a child with more than SKEW_FACTOR times its
            // share of the parent's rows under this digit (and more than a leaf
            // holds) is crowded, except below a pivot split (those go radix).
            auto emit_child = [&](uint32_t gi, const ChildRec& cr, uint64_t r0, uint64_t s0) {
                const GroupDesc& g0 = groups[gi];
                const Seg& par = segs[gseg[gi]];
                const uint32_t seg_kb = plan[gseg[gi]].kb_out;
                Seg c;
                c.buf = dst;
                c.kb = seg_kb;
                c.r0 = r0;
                c.rn = cr.rn;
                c.s0 = s0;
                c.sn = cr.sn;
                c.lo = cr.lo;
                c.hi = cr.hi;
                c.win = par.win;
                c.koff_r = g0.dst_koff;
                c.koff_s = nside == 2 ? groups[gi + 1].dst_koff : 0;
                c.wdisp = par.wdisp;
                c.wdisp_s = par.wdisp_s;
                const uint64_t rows = c.rn + c.sn, share = (par.rn + par.sn) >> g0.bits;
                c.skew = !(g0.flags & GROUP_PIVOT) && c.lo < c.hi && rows > (uint64_t)LEAF_CAP &&
                         rows > SKEW_FACTOR * share;
                if (seg_kb < kb_in && c.lo <= c.hi) {
                    // keys now hold (ord - g.base) mod 2^32 (see k_scatter)
                    const uint64_t off = c.lo - g0.base;
                    c.win = g0.base + (off & ~0xffffffffull);
                    c.lo = off & 0xffffffffull;
                    c.hi = (c.hi - g0.base) & 0xffffffffull;
                }
                sink(c);
            };
            TJ_CK(launch_children(d_groups, ng, nside, d_ccount, d_gmin, d_gmax, d_crec, st));
            // device leaves of a range share one key width (one leaf launch)
            if (dev_ok && (mixed || (dev_leaves && dev_kb != kb_out))) TJ_RET(demote_device_leaves());
            if (dev_ok) {
                // Batch the children into leaves on the device; the host reads back
                // four summary words and the children too large for a leaf.
                BatchArgs ba{};
                ba.nseg = ng / (uint32_t)nside;
                ba.nside = (uint32_t)nside;
                ba.narrowing = kb_out < kb_in ? 1u : 0u;
                ba.join = sh.join ? 1u : 0u;
                ba.buf = dst;
                ba.kb = kb_out;
                ba.flags = (g_debug_flags.load() & TJ_DEBUG_FORCE_REORDER) ? LEAF_FORCE_REORDER : 0u;
                ba.leaf_base = dev_leaves;
                ba.leaf_cap = caps.leaves;
                ba.out_delta = cur_out_delta;
                uint64_t* d_sum = d_probe + 4;  // [3] (the range-miss word) is cleared with them
                TJ_CK(launch_fill_u64(d_sum, 5, 0, st));
                TJ_CK(launch_batch_leaves(d_groups, d_crec, ba, d_segcount, d_leaves, d_sum, 0, st));
                TJ_CK(launch_batch_leaves(d_groups, d_crec, ba, d_segcount, d_leaves, d_sum, 1, st));
                uint64_t* pin = (uint64_t*)pinned_down(5 * sizeof(uint64_t));
                if (!pin) return TJ_E_HIP;
                TJ_CK(hipMemcpyAsync(pin, d_sum, 5 * sizeof(uint64_t), hipMemcpyDeviceToHost, st));
                TJ_CK(hipStreamSynchronize(st));
                const uint64_t sum[5] = {pin[0], pin[1], pin[2], pin[3], pin[4]};
                const uint64_t nbig = sum[4];
                if (!(sum[2] & BATCH_OVERFLOW) && dev_leaves + sum[0] + nbig <= caps.leaves) {
                    stats.bytes_written += written;
                    dev_leaves += (uint32_t)sum[0];
                    dev_rows += sum[1];
                    dev_wide = dev_wide || (sum[2] & BATCH_WIDE);
                    dev_kb = kb_out;
                    if (nbig == 0) continue;
                    // The listed children (slot caps.leaves - 1 - k for the k-th)
                    // go to the sink; the leaves batched so far move to the host
                    // list first, which later levels then extend.
                    BigChild* big = (BigChild*)pinned_down((size_t)nbig * sizeof(LeafDesc));
                    if (!big) return TJ_E_HIP;
                    TJ_CK(hipMemcpyAsync(big, d_leaves + (caps.leaves - nbig), (size_t)nbig * sizeof(LeafDesc),
                                         hipMemcpyDeviceToHost, st));
                    TJ_CK(hipStreamSynchronize(st));
                    std::vector<BigChild>& bl = hv.big;
                    bl.resize(nbig);
                    for (uint64_t k = 0; k < nbig; k++)
                        bl[k] = *(const BigChild*)((const LeafDesc*)big + (nbig - 1 - k));
                    TJ_RET(demote_device_leaves());
                    HostTimer ht(this, F_HOST_CLASSIFY);
                    for (const BigChild& b : bl) {
                        const uint32_t gi = b.seg * (uint32_t)nside;
                        if (b.seg >= ng / (uint32_t)nside) return TJ_E_INTERNAL;
                        const ChildRec cr{b.rn, b.sn, b.lo, b.hi};
                        emit_child(gi, cr, groups[gi].dst_start + b.r_off,
                                   nside == 2 ? groups[gi + 1].dst_start + b.s_off : 0);
                    }
                    continue;
                }
                TJ_RET(demote_device_leaves());  // this level needs the host planner
            }
            ChildRec* rec = (ChildRec*)pinned_down((size_t)nrec * sizeof(ChildRec));
            if (!rec) return TJ_E_HIP;
            TJ_CK(hipMemcpyAsync(rec, d_crec, nrec * sizeof(ChildRec), hipMemcpyDeviceToHost, st));
            TJ_CK(hipStreamSynchronize(st));
            // children in key order: segment order, then digit order; a child's
            // rows start where its smaller-digit siblings end
            HostTimer ht(this, F_HOST_CLASSIFY);
            if (learned) {
                // buckets over twice the mean (they take further radix passes)
                uint64_t rows = 0;
                for (uint32_t i = 0; i < nrec; i++) rows += rec[i].rn + rec[i].sn;
                for (uint32_t i = 0; i < nrec; i++)
                    if ((uint64_t)(rec[i].rn + rec[i].sn) * nrec > 2 * rows) stats.learned_overflow++;
            }
            for (uint32_t gi = 0; gi < ng; gi += (uint32_t)nside) {
                const GroupDesc& g0 = groups[gi];
                const uint32_t nbins = 1u << g0.bits;
                const ChildRec* cr = rec + g0.child0 / (uint32_t)nside;
                uint64_t r0 = g0.dst_start, s0 = nside == 2 ? groups[gi + 1].dst_start : 0;
                for (uint32_t d = 0; d < nbins; d++) {
                    if (cr[d].rn == 0 && cr[d].sn == 0) continue;  // no rows: every sink ignores it
                    emit_child(gi, cr[d], r0, s0);
                    r0 += cr[d].rn;
                    s0 += cr[d].sn;
                }
            }
            stats.bytes_written += written;
        }
        return TJ_OK;
    }

    // ---- pivot choice for crowded buckets ----------------------------------
    // A crowded bucket (Seg::skew) is usually crowded by one frequent key. A
    // radix digit separates that key from its neighbours only as fast as the
    // digit narrows the key range, one level at a time; a split around the key
    // itself (GROUP_PIVOT: below, equal, above) isolates it in one pass as a
    // single-key bucket. The key is taken when at least two of three rows
    // sampled at the start, middle and end of the bucket's larger side hold it;
    // otherwise the bucket takes its radix digit. Either way the result is the
    // same: the split only changes how many passes the bucket takes.
    template <class PlanVec>
    int pick_pivots(const std::vector<Seg>& segs, PlanVec& plan)
    {
        std::vector<size_t> who;
        const size_t most = std::min<size_t>(MAX_PIVOT_SEGS, caps.children / 3);
        for (size_t i = 0; i < segs.size() && who.size() < most; i++) {
            plan[i].pivot = false;
            const Seg& s = segs[i];
            // (a Seg's rows sit at r0 / s0 of its own buffer, window or not)
            if (s.skew && s.buf != BUF_IN) who.push_back(i);
        }
        if (who.empty()) return TJ_OK;
        std::vector<KeyRef> refs(3 * who.size());
        for (size_t j = 0; j < who.size(); j++) {
            const Seg& s = segs[who[j]];
            const int side = s.sn > s.rn ? 1 : 0;
            const uint64_t r0 = side ? s.s0 : s.r0, n = side ? s.sn : s.rn;
            const uint64_t koff = side ? s.koff_s : s.koff_r;
            const char* keys = (const char*)bufs.key[s.buf][side];
            const uint64_t at[3] = {0, n / 2, n - 1};
            for (int t = 0; t < 3; t++) refs[3 * j + t] = KeyRef{keys + (r0 + at[t] + koff) * s.kb, s.kb, 0};
        }
        // the child records' table is free between passes
        const uint32_t m = (uint32_t)refs.size();
        KeyRef* d_refs = (KeyRef*)d_crec;
        uint64_t* d_out = (uint64_t*)(d_refs + m);
        uint64_t* got = (uint64_t*)pinned_down((size_t)m * 8);
        if (!got) return TJ_E_HIP;
        TJ_CK(upload(d_refs, refs.data(), (size_t)m * sizeof(KeyRef), st, 1));
        TJ_CK(launch_read_ords(d_refs, m, d_out, st));
        TJ_CK(hipMemcpyAsync(got, d_out, (size_t)m * 8, hipMemcpyDeviceToHost, st));
        TJ_CK(hipStreamSynchronize(st));
        for (size_t j = 0; j < who.size(); j++) {
            const uint64_t a = got[3 * j], b = got[3 * j + 1], c = got[3 * j + 2];
            const bool ab = a == b, ac = a == c, bc = b == c;
            if (!(ab || ac || bc)) continue;
            plan[who[j]].pivot = true;
            plan[who[j]].key = ab || ac ? a : b;
            stats.pivots++;
        }
        return TJ_OK;
    }

    // ---- classification and leaf batching of buckets ----------------------
    // Buckets arrive in key order, one level at a time. Those that need another
    // pass go to `next`; the rest become leaves (adjacent small buckets batched
    // up to LEAF_CAP rows), crosses (join) or copies (sort). `out_delta` maps
    // buffer rows to output rows of the sort. classify_flush closes the open
    // leaf at the end of a level.
    // Leaves batched on the device for the current key range: d_leaves[0, dev_leaves).
    // Used for a level only when no host-side leaf, cross or copy exists yet
    // (so that the device leaves are the range's leaves in key order).
    bool dev_ok = false;
    uint32_t dev_leaves = 0, dev_kb = 0;
    uint64_t dev_rows = 0;
    bool dev_wide = false;
    uint64_t cur_out_delta = 0;

    // Moves the device leaves to the host list (they precede every later leaf).
    int demote_device_leaves()
    {
        if (dev_leaves) {
            const size_t n0 = leaves.size();
            leaves.resize(n0 + dev_leaves);
            TJ_CK(hipMemcpyAsync(leaves.data() + n0, d_leaves, (size_t)dev_leaves * sizeof(LeafDesc),
                                 hipMemcpyDeviceToHost, st));
            TJ_CK(hipStreamSynchronize(st));
            if (sh.join)  // the device leaves the join's `out` at 0: set its key-order position
                for (size_t i = n0; i < leaves.size(); i++) leaves[i].out = leaves[i].r0;
        }
        dev_leaves = 0;
        dev_rows = 0;
        dev_wide = false;
        dev_ok = false;
        return TJ_OK;
    }

    bool cl_open = false, cl_useful = false;
    int64_t cl_wdisp = 0, cl_wdisp_s = 0;
    LeafDesc cl_cur{};
    uint64_t cl_lo = 0, cl_hi = 0, cl_win = 0;
    uint32_t cl_kb = 0;

    void classify_flush(uint64_t out_delta)
    {
        if (cl_open && cl_useful) {
            cl_cur.base = cl_lo;
            cl_cur.bits = (uint16_t)nbits64(cl_hi - cl_lo);
            cl_cur.kb = (uint16_t)cl_kb;
            cl_cur.flags = (g_debug_flags.load() & TJ_DEBUG_FORCE_REORDER) ? LEAF_FORCE_REORDER : 0;
            // sort: output row; join: key-order position (row in buffer A), the
            // order finish_join takes units in before it reuses the field
            cl_cur.out = (sh.join ? cl_cur.r0 : cl_cur.r0 + out_delta) - (cl_cur.buf == BUF_B ? cl_wdisp : 0);
            leaves.push_back(cl_cur);
        }
        cl_open = false;
        cl_useful = false;
    }

    void classify_one(const Seg& s, std::vector<Seg>& next, uint64_t out_delta)
    {
        const uint64_t rows = s.rn + s.sn;
        if (rows == 0) return;  // occupies no rows: does not break adjacency
        const bool single = s.lo == s.hi;
        const bool both = s.rn > 0 && s.sn > 0;
        const bool useful = sh.join ? both : true;
        if (rows <= (uint64_t)LEAF_CAP) {
            const bool adjacent = cl_open && cl_cur.buf == s.buf && cl_kb == s.kb && cl_win == s.win &&
                                  cl_cur.kr0 - cl_cur.r0 == s.koff_r && cl_cur.ks0 - cl_cur.s0 == s.koff_s &&
                                  cl_cur.r0 + cl_cur.rn == s.r0 && cl_wdisp == s.wdisp && cl_wdisp_s == s.wdisp_s &&
                                  (!sh.join || cl_cur.s0 + cl_cur.sn == s.s0) &&
                                  cl_cur.rn + cl_cur.sn + rows <= (uint64_t)LEAF_CAP;
            if (!adjacent) {
                classify_flush(out_delta);
                cl_open = true;
                cl_cur = LeafDesc{};
                cl_cur.r0 = s.r0;
                cl_cur.s0 = s.s0;
                cl_cur.kr0 = s.r0 + s.koff_r;
                cl_cur.ks0 = s.s0 + s.koff_s;
                cl_cur.buf = (uint16_t)s.buf;
                cl_lo = s.lo;
                cl_hi = s.hi;
                cl_kb = s.kb;
                cl_win = s.win;
                cl_wdisp = s.wdisp;
                cl_wdisp_s = s.wdisp_s;
            }
            cl_cur.rn += (uint32_t)s.rn;
            cl_cur.sn += (uint32_t)s.sn;
            cl_lo = std::min(cl_lo, s.lo);
            cl_hi = std::max(cl_hi, s.hi);
            cl_useful = cl_useful || useful;
            return;
        }
        classify_flush(out_delta);
        if (sh.join && !both) return;  // no partner rows: no output
        if (single) {
            stats.single_key++;
            if (sh.join) {
                CrossDesc c{};
                c.r0 = s.r0;
                c.s0 = s.s0;
                c.a = s.rn;
                c.b = s.sn;
                c.buf = s.buf;
                c.out = s.r0 - (s.buf == BUF_B ? s.wdisp : 0);  // key-order position (see classify_flush)
                crosses.push_back(c);
            } else if (!(out_is_a && s.buf == BUF_A && out_delta == a_off)) {
                CopyDesc c{};
                c.start = s.r0;
                c.len = s.rn;
                c.out = s.r0 + out_delta - (s.buf == BUF_B ? s.wdisp : 0);
                c.buf = s.buf;
                copies.push_back(c);
            }
            return;
        }
        next.push_back(s);
    }

    // ---- learned partitioner: fit d_model to a sample of the key columns ----
    // Gathers the sample of a (and of b, when nb > 0), sorts it with the plain
    // sort path and runs the fit kernels, all inside scratch[0, scratch_bytes)
    // (device memory nothing else uses meanwhile). TJ_E_WORKSPACE when the
    // scratch cannot hold the sample and the sort's smallest workspace.
    int train_rmi(const void* a, uint64_t na, const void* b, uint64_t nb, uint32_t permille, char* scratch,
                  uint64_t scratch_bytes)
    {
        const uint64_t ma = rmi_sample_rows(na, permille), mb = nb ? rmi_sample_rows(nb, permille) : 0;
        const uint64_t M = ma + mb;
        if (M == 0 || M > kMaxRows) return TJ_E_ARG;
        char* p = scratch;
        char* end = scratch + scratch_bytes;
        auto take = [&](uint64_t bytes) -> char* {
            char* q = p;
            p += align_up(bytes, ALIGN);
            return q;
        };
        const int kb = sh.kb;
        char* skeys = take(M * kb);
        int32_t* srids = (int32_t*)take(M * 4);
        char* okeys = take(M * kb);
        int32_t* orids = (int32_t*)take(M * 4);
        uint32_t* start = (uint32_t*)take((TJ_RMI_LEAVES + 1) * 4);
        if (p >= end) return TJ_E_WORKSPACE;
        int rc = TJ_OK;
        const hipError_t e = timed(F_RMI_TRAIN, M * (uint64_t)(2 * kb + 8), [&]() -> hipError_t {
            hipError_t h = launch_rmi_sample(kb, a, na, (uint32_t)ma, skeys, srids, 0, st);
            if (h == hipSuccess && mb) h = launch_rmi_sample(kb, b, nb, (uint32_t)mb, skeys, srids, (uint32_t)ma, st);
            if (h != hipSuccess) return h;
            t_nested++;
            rc = tj_sort(kb, skeys, srids, M, okeys, orids, p, (uint64_t)(end - p), st, nullptr);
            t_nested--;
            if (rc != TJ_OK) return hipSuccess;
            return launch_rmi_fit(kb, okeys, (uint32_t)M, LEARNED_BUCKETS, start, d_model, st);
        });
        if (rc != TJ_OK) return rc;
        TJ_CK(e);
        stats.sample_rows = M;
        stats.bytes_read += M * (uint64_t)kb;
        return TJ_OK;
    }

    // ---- process one key range (the whole domain when the budget does not bind)
    int process_range(uint64_t lo, uint64_t hi, uint64_t rn, uint64_t sn, bool filtered,
                      uint64_t out_delta)
    {
        Seg root{};
        root.kb = (uint32_t)sh.kb;
        root.r0 = 0;
        root.rn = rn;
        root.s0 = 0;
        root.sn = sn;
        root.lo = lo;
        root.hi = hi;
        root.buf = BUF_IN;
        std::vector<Seg> next, next2;
        auto to_next = [&](const Seg& c) { classify_one(c, next, out_delta); };
        cur_out_delta = out_delta;
        auto allow_device = [&]() {
            dev_ok = device_batching && leaves.empty() && crosses.empty() && copies.empty() && dev_leaves == 0;
        };
        if (filtered) {
            // first pass: compaction + split of the range's rows out of the input
            const uint64_t f[2] = {lo, hi};
            std::vector<Seg> roots{root};
            allow_device();
            TJ_RET(run_pass(roots, BUF_IN, BUF_A, f, to_next));
            dev_ok = false;
        } else {
            classify_one(root, next, out_delta);
        }
        classify_flush(out_delta);
        if (filtered && window && !next.empty()) {
            // The buckets that need further passes are packed one after
            // another into the window. While they do not fit, the largest is
            // read again from the input, filtered to its key range, into its
            // own rows of A with a full digit of that narrower range (its keys
            // are still there): its children replace it.
            for (int it = 0;; it++) {
                uint64_t ur = 0, us = 0;
                size_t big = 0;
                for (size_t i = 0; i < next.size(); i++) {
                    ur += next[i].rn;
                    us += next[i].sn;
                    if (next[i].rn * win_s + next[i].sn * win_r > next[big].rn * win_s + next[big].sn * win_r) big = i;
                }
                if (ur <= win_r && us <= win_s) break;
                if (it >= 4096) return TJ_E_INTERNAL;
                const Seg c = next[big];
                next.erase(next.begin() + (std::ptrdiff_t)big);
                Seg again{};
                again.kb = (uint32_t)sh.kb;
                again.r0 = c.r0;
                again.rn = c.rn;
                again.s0 = c.s0;
                again.sn = c.sn;
                again.lo = c.win == ~0ull ? c.lo : c.win + c.lo;  // ordinals of the input keys
                again.hi = c.win == ~0ull ? c.hi : c.win + c.hi;
                again.buf = BUF_IN;
                std::vector<Seg> roots{again};
                const uint64_t f[2] = {again.lo, again.hi};
                stats.key_ranges++;  // one more read of the inputs
                TJ_RET(run_pass(roots, BUF_IN, BUF_A, f, to_next));
                classify_flush(out_delta);
            }
            uint64_t ur = 0, us = 0;
            for (Seg& g : next) {
                g.wdisp = (int64_t)ur - (int64_t)g.r0;
                g.wdisp_s = (int64_t)us - (int64_t)g.s0;
                ur += g.rn;
                us += g.sn;
            }
            stats.windows++;
        }
        uint32_t cur = filtered ? (uint32_t)BUF_A : (uint32_t)BUF_IN;
        for (int depth = 0; depth < 80; depth++) {
            if (next.empty()) return TJ_OK;
            const uint32_t dst = cur == BUF_A ? (uint32_t)BUF_B : (uint32_t)BUF_A;
            next2.clear();
            allow_device();
            TJ_RET(run_pass(next, cur, dst, nullptr, [&](const Seg& c) { classify_one(c, next2, out_delta); }));
            dev_ok = false;
            classify_flush(out_delta);
            next.swap(next2);
            cur = dst;
        }
        return TJ_E_INTERNAL;
    }

    // Leaves of buffer A (the output columns from row a_off) wait for the
    // end of the call in `deferred`; the others (in the window, or read from
    // the input) are sorted now, before their rows can be overwritten.
    int run_window_leaves(void* out_k, int32_t* out_r)
    {
        size_t keep = 0;
        for (size_t i = 0; i < leaves.size(); i++) {
            LeafDesc L = leaves[i];
            if (L.buf == BUF_A) {
                L.r0 += a_off;
                L.kr0 += a_off;
                deferred.push_back(L);
            } else {
                leaves[keep++] = L;
            }
        }
        leaves.resize(keep);
        return run_sort_leaves(out_k, out_r);
    }

    // ---- sort under a binding budget: output columns plus a window ---------
    // Sorts the `rows` rows with keys in [lo, hi] into output rows [o, o +
    // rows). Buffer A is the output columns from row o. The first pass reads
    // the input (`filtered`: keeping only the rows in [lo, hi], which the
    // input still holds) and partitions them straight into A, where buckets
    // that are leaves are sorted in place and single-key buckets are already
    // final. Buckets that need more passes take them through the workspace
    // window (buffer B, wrows rows at wk / wr): a run of buckets (in key
    // order) at a time, packed one after another into the window (each with
    // its own Seg::wdisp), ping-ponging between their own rows of A and their
    // place in the window until every child is a leaf; each run's leaves are
    // sorted before the window moves on. A bucket of more than wrows rows is
    // sorted the same way into its own rows of A, from the input filtered to
    // its key range.
    int sort_windowed(uint64_t lo, uint64_t hi, uint64_t rows, uint64_t o, bool filtered, int depth, void* out_k,
                      int32_t* out_r, char* wk, char* wr, uint64_t wrows)
    {
        if (depth > 64) return TJ_E_INTERNAL;
        bufs.key[BUF_A][0] = (char*)out_k + o * (uint64_t)sh.kb;
        bufs.rid[BUF_A][0] = out_r + o;
        a_off = o;
        Seg root{};
        root.kb = (uint32_t)sh.kb;
        root.rn = rows;
        root.lo = lo;
        root.hi = hi;
        root.buf = BUF_IN;
        std::vector<Seg> next, level, next2, big;
        auto allow_device = [&]() {
            dev_ok = device_batching && leaves.empty() && crosses.empty() && copies.empty() && dev_leaves == 0;
        };
        cur_out_delta = o;
        if (filtered) {
            const uint64_t f[2] = {lo, hi};
            next.push_back(root);
            stats.key_ranges++;  // one more read of the input
            allow_device();
            TJ_RET(run_pass(next, BUF_IN, BUF_A, f, [&](const Seg& c) { classify_one(c, level, o); }));
            dev_ok = false;
        } else {
            classify_one(root, next, o);
            classify_flush(o);
            if (!next.empty()) {
                allow_device();
                TJ_RET(run_pass(next, BUF_IN, BUF_A, nullptr, [&](const Seg& c) { classify_one(c, level, o); }));
                dev_ok = false;
            }
        }
        classify_flush(o);
        TJ_RET(run_window_leaves(out_k, out_r));
        size_t i = 0;
        while (i < level.size()) {
            if (level[i].rn > wrows) {
                big.push_back(level[i++]);
                continue;
            }
            // pack a run of buckets into the window, each at its own offset
            next.clear();
            uint64_t used = 0;
            while (i < level.size() && level[i].rn <= wrows && used + level[i].rn <= wrows) {
                Seg g = level[i++];
                g.wdisp = (int64_t)used - (int64_t)g.r0;
                used += g.rn;
                next.push_back(g);
            }
            bufs.key[BUF_B][0] = wk;
            bufs.rid[BUF_B][0] = (const int32_t*)wr;
            stats.windows++;
            uint32_t cur = BUF_A;
            for (int d = 0; !next.empty(); d++) {
                if (d >= 80) return TJ_E_INTERNAL;
                const uint32_t dst = cur == BUF_A ? (uint32_t)BUF_B : (uint32_t)BUF_A;
                next2.clear();
                allow_device();
                TJ_RET(run_pass(next, cur, dst, nullptr, [&](const Seg& c) { classify_one(c, next2, o); }));
                dev_ok = false;
                classify_flush(o);
                next.swap(next2);
                cur = dst;
            }
            TJ_RET(run_window_leaves(out_k, out_r));
        }
        for (const Seg& b : big)
            TJ_RET(sort_windowed(b.lo, b.hi, b.rn, o + b.r0, true, depth + 1, out_k, out_r, wk, wr, wrows));
        if (depth == 0 && !deferred.empty()) {
            // the leaves already in the output columns, all in one launch
            bufs.key[BUF_A][0] = out_k;
            bufs.rid[BUF_A][0] = out_r;
            a_off = 0;
            leaves.swap(deferred);
            deferred.clear();
            TJ_RET(run_sort_leaves(out_k, out_r));
        }
        return TJ_OK;
    }

    // ---- leaves and singles ---------------------------------------------
    int run_sort_leaves(void* out_k, int32_t* out_r)
    {
        if (dev_leaves) {
            // batched on the device: no other leaf or copy exists in this range
            if (!leaves.empty() || !copies.empty()) return TJ_E_INTERNAL;
            const uint32_t n = dev_leaves;
            TJ_CK(timed(F_LEAF_SORT, dev_rows * row_bytes(sh.kb, true) * 2, [&] {
                return launch_leaf_sort(sh.kb, dev_wide, d_leaves, n, bufs, out_k, out_r, st);
            }));
            TJ_CK(hipStreamSynchronize(st));
            stats.leaves += n;
            stats.bytes_read += dev_rows * row_bytes(sh.kb, true);
            stats.bytes_written += dev_rows * row_bytes(sh.kb, true);
            dev_leaves = 0;
            dev_rows = 0;
            dev_wide = false;
            return TJ_OK;
        }
        HostTimer ht(this, F_HOST_LEAVES);
        for (int wide = 0; wide < 2; wide++) {
            std::vector<LeafDesc>& sel = hv.batch_leaves;
            sel.clear();
            for (const LeafDesc& L : leaves)
                if ((L.bits > 32) == (wide == 1)) sel.push_back(L);
            ht.stop();
            for (size_t i = 0; i < sel.size(); i += caps.leaves) {
                const uint32_t n = (uint32_t)std::min<size_t>(caps.leaves, sel.size() - i);
                TJ_CK(upload(d_leaves, sel.data() + i, n * sizeof(LeafDesc), st, 0));
                uint64_t rows = 0;
                for (uint32_t k = 0; k < n; k++) rows += sel[i + k].rn;
                TJ_CK(timed(F_LEAF_SORT, rows * row_bytes(sh.kb, true) * 2, [&] {
                    return launch_leaf_sort(sh.kb, wide == 1, d_leaves, n, bufs, out_k, out_r, st);
                }));
                TJ_CK(hipStreamSynchronize(st));
            }
        }
        stats.leaves += (uint32_t)leaves.size();
        for (const LeafDesc& L : leaves) {
            stats.bytes_read += L.rn * row_bytes(sh.kb, true);
            stats.bytes_written += L.rn * row_bytes(sh.kb, true);
        }
        // copies
        for (size_t i = 0; i < copies.size(); i += caps.units) {
            const uint32_t n = (uint32_t)std::min<size_t>(caps.units, copies.size() - i);
            uint64_t t = 0;
            for (uint32_t k = 0; k < n; k++) {
                copies[i + k].pfx = t;
                t += copies[i + k].len;
            }
            stats.bytes_read += t * row_bytes(sh.kb, true);
            stats.bytes_written += t * row_bytes(sh.kb, true);
            TJ_CK(hipMemcpyAsync(d_units, copies.data() + i, n * sizeof(CopyDesc), hipMemcpyHostToDevice, st));
            TJ_CK(timed(F_COPY, t * row_bytes(sh.kb, true) * 2, [&] {
                return launch_copy(sh.kb, (const CopyDesc*)d_units, n, t, bufs, out_k, out_r, st);
            }));
            TJ_CK(hipStreamSynchronize(st));
        }
        leaves.clear();
        copies.clear();
        return TJ_OK;
    }

    // Counts (mat = false) or materialises (mat = true) the range's leaves and
    // crosses. Units are taken in key order, which is the order of their first
    // R row (every unit has R rows, and partitioning keeps each bucket inside
    // its parent's index range). Output starts at `base`; pairs at or beyond
    // `capacity` are not written. *total_out receives the range's pair count.
    int finish_join(uint64_t* total_out, uint64_t base, int32_t* out_r, int32_t* out_s,
                    uint64_t capacity, bool mat)
    {
        if (dev_leaves) {
            // batched on the device: no other leaf or cross exists in this range
            if (!leaves.empty() || !crosses.empty()) return TJ_E_INTERNAL;
            const uint32_t nl = dev_leaves;
            const int kb = (int)dev_kb;
            const bool wide = dev_wide;
            const uint64_t rows = dev_rows;
            dev_leaves = 0;
            dev_rows = 0;
            dev_wide = false;
            stats.leaves += nl;
            uint64_t* d_total = d_probe + 2;
            uint32_t* d_ticket = (uint32_t*)(d_probe + 3);
            uint32_t* d_err = d_ticket + 1;
            if (!mat) {
                TJ_CK(launch_fill_u64(d_total, 1, 0, st));
                TJ_CK(timed(F_LEAF_COUNT, rows * kb, [&] {
                    return launch_leaf_join(kb, wide, false, d_leaves, nl, bufs, d_status, d_ticket, d_total,
                                            d_err, nullptr, nullptr, 0, st);
                }));
                uint64_t t = 0;
                TJ_CK(hipMemcpyAsync(&t, d_total, 8, hipMemcpyDeviceToHost, st));
                TJ_CK(hipStreamSynchronize(st));
                stats.bytes_read += rows * kb;
                *total_out = t;
                return TJ_OK;
            }
            TJ_CK(launch_fill_u64(d_status, 1, STATUS_INCLUSIVE | base, st));
            TJ_CK(launch_fill_u64(d_status + 1, nl, 0, st));
            TJ_CK(launch_fill_u64(d_probe + 3, 1, 0, st));  // ticket and error flag
            const size_t leaf_timer = pending.size();
            TJ_CK(timed(F_LEAF_MAT, rows * row_bytes(kb, true), [&] {
                return launch_leaf_join(kb, wide, true, d_leaves, nl, bufs, d_status, d_ticket, d_total, d_err,
                                        out_r, out_s, capacity, st);
            }));
            stats.bytes_read += rows * row_bytes(kb, true);
            uint64_t fin[2] = {0, 0};
            TJ_CK(hipMemcpyAsync(&fin[0], d_status + nl, 8, hipMemcpyDeviceToHost, st));
            TJ_CK(hipMemcpyAsync(&fin[1], d_probe + 3, 8, hipMemcpyDeviceToHost, st));
            TJ_CK(hipStreamSynchronize(st));
            if (fin[1] >> 32) return TJ_E_INTERNAL;  // a look-back expired
            const uint64_t end = fin[0] & STATUS_VALUE;
            if (leaf_timer < pending.size()) pending[leaf_timer].bytes += (end - base) * 8;
            *total_out = end - base;
            const uint64_t written = std::min(end, capacity) > base ? std::min(end, capacity) - base : 0;
            stats.bytes_written += written * 8;
            return TJ_OK;
        }
        HostTimer ht(this, F_HOST_LEAVES);
        stats.leaves += (uint32_t)leaves.size();
        uint64_t* d_total = d_probe + 2;
        uint32_t* d_ticket = (uint32_t*)(d_probe + 3);
        uint32_t* d_err = d_ticket + 1;
        if (!mat) {
            uint64_t cross_pairs = 0;
            for (const CrossDesc& c : crosses) cross_pairs += c.a * c.b;
            ht.stop();
            TJ_CK(launch_fill_u64(d_total, 1, 0, st));
            // leaves grouped by key width (order does not matter for a count)
            for (int kb : {8, 4}) {
                std::vector<LeafDesc>& sel = hv.batch_leaves;
                sel.clear();
                for (size_t i = 0; i < leaves.size(); i++)
                    if (leaves[i].kb == kb) sel.push_back(leaves[i]);
                for (size_t i = 0; i < sel.size(); i += caps.leaves) {
                    const uint32_t n = (uint32_t)std::min<size_t>(caps.leaves, sel.size() - i);
                    uint64_t rows = 0;
                    bool wide = false;
                    for (uint32_t k = 0; k < n; k++) {
                        rows += sel[i + k].rn + sel[i + k].sn;
                        wide = wide || sel[i + k].bits > 32;
                    }
                    TJ_CK(upload(d_leaves, sel.data() + i, n * sizeof(LeafDesc), st, 0));
                    TJ_CK(timed(F_LEAF_COUNT, rows * kb, [&] {
                        return launch_leaf_join(kb, wide, false, d_leaves, n, bufs, d_status, d_ticket, d_total,
                                                d_err, nullptr, nullptr, 0, st);
                    }));
                    stats.bytes_read += rows * kb;
                    // the selection buffer is refilled for the next width: wait for the upload
                    TJ_CK(hipStreamSynchronize(st));
                }
            }
            uint64_t t = 0;
            TJ_CK(hipMemcpyAsync(&t, d_total, 8, hipMemcpyDeviceToHost, st));
            TJ_CK(hipStreamSynchronize(st));
            *total_out = t + cross_pairs;
        } else {
            // Key order of the units is the order of their R rows in buffer A
            // (LeafDesc/CrossDesc::out until batched). Leaves of a level are
            // appended in that order, deeper levels after: order (position,
            // index) pairs, a stable LSD radix sort, and read the leaves through them.
            const std::vector<std::pair<uint64_t, uint32_t>>* ord = nullptr;
            if (!std::is_sorted(leaves.begin(), leaves.end(),
                                [](const LeafDesc& a, const LeafDesc& b) { return a.out < b.out; })) {
                auto& o = hv.order;
                o.resize(leaves.size());
                uint64_t top = 0;
                for (size_t i = 0; i < leaves.size(); i++) {
                    o[i] = {leaves[i].out, (uint32_t)i};
                    top = std::max(top, leaves[i].out);
                }
                radix_order(o, hv.order_tmp, top);
                ord = &o;
            }
            auto leaf_at = [&](size_t i) -> const LeafDesc& { return ord ? leaves[(*ord)[i].second] : leaves[i]; };
            auto cr0 = [](const CrossDesc& a, const CrossDesc& b) { return a.out < b.out; };
            if (!std::is_sorted(crosses.begin(), crosses.end(), cr0)) std::sort(crosses.begin(), crosses.end(), cr0);
            uint64_t carry = base;
            size_t li = 0, ci = 0;
            std::vector<LeafDesc>& bl = hv.batch_leaves;
            std::vector<CrossDesc>& bc = hv.batch_crosses;
            while (li < leaves.size() || ci < crosses.size()) {
                bl.clear();
                bc.clear();
                uint64_t pre = 0;  // single-key pairs of this batch so far
                int bkb = 0;       // key width of the batch's leaves
                while (li < leaves.size() || ci < crosses.size()) {
                    const bool take_cross =
                        ci < crosses.size() && (li == leaves.size() || crosses[ci].out < leaf_at(li).out);
                    if (take_cross) {
                        if (bc.size() == caps.units) break;
                        CrossDesc c = crosses[ci++];
                        c.out = pre;
                        c.leaf_before = (uint32_t)bl.size();
                        c.pfx = 0;
                        pre += c.a * c.b;
                        bc.push_back(c);
                    } else {
                        if (bl.size() == caps.leaves) break;
                        if (bkb != 0 && leaf_at(li).kb != bkb) break;  // one launch, one key width
                        bkb = leaf_at(li).kb;
                        LeafDesc L = leaf_at(li++);
                        L.out = pre;
                        bl.push_back(L);
                    }
                }
                const uint32_t nl = (uint32_t)bl.size(), nc = (uint32_t)bc.size();
                ht.stop();
                TJ_CK(launch_fill_u64(d_status, 1, STATUS_INCLUSIVE | carry, st));
                TJ_CK(launch_fill_u64(d_status + 1, nl, 0, st));
                TJ_CK(launch_fill_u64(d_probe + 3, 1, 0, st));  // ticket and error flag
                size_t leaf_timer = (size_t)-1;
                if (nl) {
                    uint64_t rows = 0;
                    bool wide = false;
                    for (const LeafDesc& L : bl) {
                        rows += L.rn + L.sn;
                        wide = wide || L.bits > 32;
                    }
                    leaf_timer = pending.size();
                    TJ_CK(upload(d_leaves, bl.data(), nl * sizeof(LeafDesc), st, 0));
                    TJ_CK(timed(F_LEAF_MAT, rows * row_bytes(bkb, true), [&] {
                        return launch_leaf_join(bkb, wide, true, d_leaves, nl, bufs, d_status, d_ticket,
                                                d_total, d_err, out_r, out_s, capacity, st);
                    }));
                    stats.bytes_read += rows * row_bytes(bkb, true);
                }
                if (nc) {
                    uint64_t t = 0, in_rows = 0;
                    for (CrossDesc& c : bc) {
                        c.pfx = t;
                        t += c.a * c.b;
                        in_rows += c.a + c.b;
                    }
                    TJ_CK(upload(d_units, bc.data(), nc * sizeof(CrossDesc), st, 1));
                    TJ_CK(timed(F_CROSS, t * 8 + in_rows * 4, [&] {
                        return launch_cross((const CrossDesc*)d_units, nc, t, bufs, d_status, out_r, out_s,
                                            capacity, st);
                    }));
                    stats.bytes_read += in_rows * 4;
                }
                uint64_t fin[2] = {0, 0};
                TJ_CK(hipMemcpyAsync(&fin[0], d_status + nl, 8, hipMemcpyDeviceToHost, st));
                TJ_CK(hipMemcpyAsync(&fin[1], d_probe + 3, 8, hipMemcpyDeviceToHost, st));
                TJ_CK(hipStreamSynchronize(st));
                if (fin[1] >> 32) return TJ_E_INTERNAL;  // a look-back expired
                const uint64_t leaf_pairs = (fin[0] & STATUS_VALUE) - carry;
                if (leaf_timer < pending.size()) pending[leaf_timer].bytes += leaf_pairs * 8;
                carry = (fin[0] & STATUS_VALUE) + pre;
            }
            *total_out = carry - base;
            const uint64_t written = std::min(carry, capacity) > base ? std::min(carry, capacity) - base : 0;
            stats.bytes_written += written * 8;
        }
        leaves.clear();
        crosses.clear();
        return TJ_OK;
    }

    // A key range holding one key value with a rows of R and b rows of S, too
    // large for the workspace: its pairs are built in the output columns. The
    // S row ids are compacted (input order) to out_s[base, base+b), the R row
    // ids to scratch space inside the pair range, then expanded R-major.
    int single_key_pairs(uint64_t k, uint64_t a, uint64_t b, uint64_t base, int32_t* out_r,
                         int32_t* out_s)
    {
        BufSet saved = bufs;
        const bool saved_wk = write_keys;
        write_keys = false;
        auto compact = [&](int side, int32_t* dst) -> int {
            bufs.rid[BUF_A][side] = dst;
            Seg root{};
            root.kb = (uint32_t)sh.kb;
            root.lo = root.hi = k;
            root.buf = BUF_IN;
            if (side == 0) root.rn = a; else root.sn = b;
            std::vector<Seg> roots{root};
            const uint64_t f[2] = {k, k};
            // only the requested side is scanned: zero the other's input length
            const uint64_t keep_r = sh.n_r, keep_s = sh.n_s;
            const bool keep_join = sh.join;
            if (side == 0) { sh.join = false; }
            else {
                // run the S column as the single side of a one-relation pass
                sh.join = false;
                bufs.key[BUF_IN][0] = saved.key[BUF_IN][1];
                bufs.rid[BUF_IN][0] = saved.rid[BUF_IN][1];
                bufs.rid[BUF_A][0] = dst;
                sh.n_r = keep_s;
            }
            int rc = run_pass(roots, BUF_IN, BUF_A, f, [](const Seg&) {});  // children unused
            sh.n_r = keep_r;
            sh.n_s = keep_s;
            sh.join = keep_join;
            bufs = saved;
            return rc;
        };
        int rc = TJ_OK;
        if (b == 1) {
            rc = compact(0, out_r + base);
            if (rc == TJ_OK) rc = compact(1, out_s + base);
            if (rc == TJ_OK && a > 1) rc = launch_expand(out_s + base, nullptr, a, 1, 1, st) == hipSuccess ? TJ_OK : TJ_E_HIP;
        } else if (a == 1) {
            rc = compact(1, out_s + base);
            if (rc == TJ_OK) rc = compact(0, out_r + base);
            if (rc == TJ_OK) rc = launch_expand(out_r + base, out_r + base, b, b, 0, st) == hipSuccess ? TJ_OK : TJ_E_HIP;
        } else {
            rc = compact(1, out_s + base);
            if (rc == TJ_OK) rc = compact(0, out_s + base + b);  // (a-1)(b-1) >= 1: fits in [b, a*b)
            if (rc == TJ_OK)
                rc = launch_expand(out_r + base, out_s + base + b, a * b, b, 0, st) == hipSuccess ? TJ_OK : TJ_E_HIP;
            if (rc == TJ_OK) rc = launch_expand(out_s + base, nullptr, a * b, b, 1, st) == hipSuccess ? TJ_OK : TJ_E_HIP;
        }
        write_keys = saved_wk;
        bufs = saved;
        stats.single_key++;
        stats.bytes_written += a * b * 8;
        return rc;
    }

    // ---- key ranges under a binding budget ---------------------------------
    // Coarse histogram of the top bits of (ord - lo) over both inputs, cut into
    // ranges whose rows fit the buffers; a bin too large is refined by a
    // histogram of its own sub-range. Computed with the partition kernels: one
    // filtered histogram pass with a wide digit.
    int coarse_hist(uint64_t lo, uint64_t hi, uint32_t& shift, uint32_t& bits,
                    std::vector<uint64_t>& cr, std::vector<uint64_t>& cs)
    {
        const uint32_t kbits = nbits64(hi - lo);
        bits = std::min<uint32_t>(kbits, MAX_DIGIT_BITS);
        if (bits == 0) bits = 1;
        shift = kbits > bits ? kbits - bits : 0;
        const int nside = sh.join ? 2 : 1;
        std::vector<GroupDesc> groups;
        std::vector<ChunkDesc> chunks;
        const uint64_t nmax = std::max(sh.n_r, sh.n_s);
        uint64_t ch_rows = align_up((nmax + 255) / 256, PART_TILE);
        if (ch_rows < PART_TILE) ch_rows = PART_TILE;
        while ((nmax + ch_rows - 1) / ch_rows * nside > caps.chunks) ch_rows *= 2;
        uint32_t child = 0;
        for (int side = 0; side < nside; side++) {
            GroupDesc g{};
            g.len = side ? sh.n_s : sh.n_r;
            g.base = lo;
            g.flo = lo;
            g.fhi = hi;
            g.shift = shift;
            g.bits = bits;
            g.side = (uint32_t)side;
            g.src = BUF_IN;
            g.chunk0 = (uint32_t)chunks.size();
            g.child0 = child;
            child += 1u << bits;
            for (uint64_t c0 = 0; c0 < g.len; c0 += ch_rows) {
                ChunkDesc c{};
                c.start = c0;
                c.len = (uint32_t)std::min<uint64_t>(ch_rows, g.len - c0);
                c.group = (uint32_t)side;
                chunks.push_back(c);
            }
            g.nchunks = (uint32_t)chunks.size() - g.chunk0;
            groups.push_back(g);
            stats.bytes_read += g.len * (uint64_t)sh.kb;
        }
        const uint32_t nc = (uint32_t)chunks.size();
        TJ_CK(hipMemcpyAsync(d_groups, groups.data(), groups.size() * sizeof(GroupDesc), hipMemcpyHostToDevice, st));
        TJ_CK(hipMemcpyAsync(d_chunks, chunks.data(), nc * sizeof(ChunkDesc), hipMemcpyHostToDevice, st));
        TJ_CK(launch_fill_u64(d_gmin, child, ~0ull, st));
        TJ_CK(launch_fill_u64(d_gmax, child, 0ull, st));
        TJ_CK(launch_hist(sh.kb, d_chunks, nc, d_groups, bufs, d_hist, d_gmin, d_gmax, nullptr, st));
        std::vector<uint32_t> h((size_t)nc * NB);
        TJ_CK(hipMemcpyAsync(h.data(), d_hist, h.size() * 4, hipMemcpyDeviceToHost, st));
        TJ_CK(hipStreamSynchronize(st));
        const uint32_t nbins = 1u << bits;
        cr.assign(nbins, 0);
        cs.assign(nbins, 0);
        for (uint32_t c = 0; c < nc; c++) {
            std::vector<uint64_t>& dstv = chunks[c].group ? cs : cr;
            for (uint32_t d = 0; d < nbins; d++) dstv[d] += h[(size_t)c * NB + d];
        }
        return TJ_OK;
    }

    struct Range {
        uint64_t lo, hi, rn, sn;
    };

    // Splits [lo, hi] into ranges with rn <= cap_r and sn <= cap_s, or single keys.
    int plan_ranges(uint64_t lo, uint64_t hi, std::vector<Range>& out, int depth)
    {
        if (depth > 16) return TJ_E_INTERNAL;
        uint32_t shift, bits;
        std::vector<uint64_t> cr, cs;
        TJ_RET(coarse_hist(lo, hi, shift, bits, cr, cs));
        const uint32_t nbins = 1u << bits;
        auto bin_lo = [&](uint32_t d) { return lo + ((uint64_t)d << shift); };
        auto bin_hi = [&](uint32_t d) {
            // last offset of bin d, formed without passing 2^64 (the top bin of
            // a full-width key range ends exactly there)
            const uint64_t off = ((uint64_t)d << shift) + ((1ull << shift) - 1);
            return off >= hi - lo ? hi : lo + off;
        };
        bool open = false;
        Range cur{};
        for (uint32_t d = 0; d < nbins; d++) {
            if (bin_lo(d) > hi) break;
            const uint64_t r = cr[d], s = cs[d];
            if (r == 0 && s == 0) continue;
            if (r > cap_r || s > cap_s) {
                if (open) out.push_back(cur);
                open = false;
                if (shift == 0 || bin_lo(d) == bin_hi(d)) {
                    out.push_back(Range{bin_lo(d), bin_lo(d), r, s});  // a single key value
                } else {
                    TJ_RET(plan_ranges(bin_lo(d), bin_hi(d), out, depth + 1));
                }
                continue;
            }
            if (open && cur.rn + r <= cap_r && cur.sn + s <= cap_s) {
                cur.hi = bin_hi(d);
                cur.rn += r;
                cur.sn += s;
            } else {
                if (open) out.push_back(cur);
                cur = Range{bin_lo(d), bin_hi(d), r, s};
                open = true;
            }
        }
        if (open) out.push_back(cur);
        return TJ_OK;
    }
};

bool timing_enabled()
{
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    return t.on;
}

int validate_common(int key_type)
{
    if (key_type != TJ_KEY_I32 && key_type != TJ_KEY_I64) return TJ_E_ARG;
    return TJ_OK;
}

bool overlap(const void* a, uint64_t abytes, const void* b, uint64_t bbytes)
{
    if (!a || !b || abytes == 0 || bbytes == 0) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bbytes && y < x + abytes;
}

// Chooses the table tier and the data layout for a given workspace budget.
// Returns TJ_E_WORKSPACE below the minimum.
int plan_workspace(const Shape& s, uint64_t ws_bytes, int& tier, bool& unlimited, uint64_t& data_bytes)
{
    const uint64_t full_data = full_data_bytes(s);
    const uint64_t min_data = min_data_bytes(s);
    tier = -1;
    // full plan: data buffers for every row plus the largest table tier that fits
    for (int t = TABLE_TIERS - 1; t >= 0; t--)
        if (full_data + table_bytes(tier_caps(t)) <= ws_bytes) {
            tier = t;
            break;
        }
    if (tier >= 0 && (tier == TABLE_TIERS - 1 || full_data + table_bytes(tier_caps(TABLE_TIERS - 1)) > ws_bytes)) {
        unlimited = true;
        data_bytes = full_data;
        return TJ_OK;
    }
    // budget binds: tables take at most a quarter, the rest holds a key range's rows
    unlimited = false;
    for (int t = TABLE_TIERS - 1; t >= 0; t--)
        if (table_bytes(tier_caps(t)) * 4 <= ws_bytes || t == 0) {
            tier = t;
            break;
        }
    const uint64_t tb = table_bytes(tier_caps(tier));
    if (ws_bytes < tb + min_data) return TJ_E_WORKSPACE;
    data_bytes = ws_bytes - tb;
    return TJ_OK;
}

uint64_t min_workspace(const Shape& s) { return table_bytes(tier_caps(0)) + min_data_bytes(s); }

uint64_t full_workspace(const Shape& s) { return table_bytes(tier_caps(TABLE_TIERS - 1)) + full_data_bytes(s); }

// Lays out the ping-pong buffers inside the data region (keys of `kb` bytes:
// the shape's key width, or 4 for a join whose key ranges narrow them).
void layout_data(Exec& x, char* p, uint64_t data_bytes, bool unlimited, int kb)
{
    const Shape& s = x.sh;
    const int nside = s.join ? 2 : 1;
    uint64_t cap[2] = {s.n_r, s.n_s};
    x.window = false;
    if (!unlimited) {
        // split the region between the sides in proportion to their rows
        const uint64_t rb = row_bytes(kb, s.rids);
        const int nbuf = s.join ? 2 : 1;  // sort: only buffer B lives in the workspace
        const uint64_t slack = (uint64_t)ALIGN * 4 * nbuf * nside;
        const uint64_t avail = data_bytes > slack ? data_bytes - slack : 0;
        const uint64_t tot = s.n_r + (s.join ? s.n_s : 0);
        for (int side = 0; side < nside; side++) {
            const uint64_t n = side ? s.n_s : s.n_r;
            const long double frac = tot ? (long double)n / (long double)tot : 1.0L;
            cap[side] = (uint64_t)((long double)avail * frac / (long double)(rb * nbuf));
            if (cap[side] > n) cap[side] = n;
        }
    }
    x.cap_r = cap[0];
    x.cap_s = s.join ? cap[1] : 0;
    for (int buf = (s.join ? BUF_A : BUF_B); buf <= BUF_B; buf++)
        for (int side = 0; side < nside; side++) {
            x.bufs.key[buf][side] = p;
            p += align_up(cap[side] * (uint64_t)kb, ALIGN);
            if (s.rids) {
                x.bufs.rid[buf][side] = (const int32_t*)p;
                p += align_up(cap[side] * 4, ALIGN);
            }
        }
}

// Budget-bound join whose ranges hold 4-byte keys: buffer A (a key range's
// rows) takes WINDOW_A_NUM / WINDOW_DEN of the data region and buffer B the
// rest, as a window into which the range's buckets that need further passes
// are packed (Exec::window); each side in proportion to its rows.
constexpr uint64_t WINDOW_A_NUM = 7, WINDOW_DEN = 8;
void layout_join_window(Exec& x, char* p, uint64_t data_bytes)
{
    const Shape& s = x.sh;
    const uint64_t rb = row_bytes(4, s.rids);
    const uint64_t slack = (uint64_t)ALIGN * 16;
    const uint64_t avail = data_bytes > slack ? data_bytes - slack : 0;
    const uint64_t tot = s.n_r + s.n_s;
    uint64_t cap[2][2];  // [buffer A/B][side]
    for (int side = 0; side < 2; side++) {
        const uint64_t n = side ? s.n_s : s.n_r;
        const long double part = (long double)avail * (long double)n / (long double)tot / (long double)rb;
        cap[0][side] = std::min<uint64_t>(n, (uint64_t)(part * WINDOW_A_NUM / WINDOW_DEN));
        cap[1][side] = std::min<uint64_t>(n, (uint64_t)(part * (WINDOW_DEN - WINDOW_A_NUM) / WINDOW_DEN));
    }
    x.cap_r = cap[0][0];
    x.cap_s = cap[0][1];
    x.win_r = cap[1][0];
    x.win_s = cap[1][1];
    x.window = true;
    for (int b = 0; b < 2; b++)
        for (int side = 0; side < 2; side++) {
            const int buf = b ? BUF_B : BUF_A;
            x.bufs.key[buf][side] = p;
            p += align_up(cap[b][side] * 4, ALIGN);
            if (s.rids) {
                x.bufs.rid[buf][side] = (const int32_t*)p;
                p += align_up(cap[b][side] * 4, ALIGN);
            }
        }
}

int probe(Exec& x, const void* a, uint64_t na, const void* b, uint64_t nb, uint64_t& lo, uint64_t& hi)
{
    uint64_t mm[2];
    TJ_CK(x.timed(F_PROBE, (na + nb) * (uint64_t)x.sh.kb,
                  [&] { return launch_probe(x.sh.kb, a, na, b, nb, x.d_probe, x.st); }));
    TJ_CK(hipMemcpyAsync(mm, x.d_probe, 16, hipMemcpyDeviceToHost, x.st));
    TJ_CK(hipStreamSynchronize(x.st));
    x.stats.bytes_read += (na + nb) * (uint64_t)x.sh.kb;
    lo = mm[0];
    hi = mm[1];
    return TJ_OK;
}

// Digit range of a first pass from every SAMPLED_PROBE_STEP-th key instead of
// all of them: the sample's minimum is rounded down to a whole digit, so rows
// a little beyond the sample's extremes still take correct digits; the first
// histogram checks every row against the range (GROUP_CHECK_RANGE).
int sampled_range(Exec& x, const void* a, uint64_t na, const void* b, uint64_t nb, uint64_t& lo, uint64_t& hi)
{
    uint64_t mm[2];
    const uint64_t sampled = (na + SAMPLED_PROBE_STEP - 1) / SAMPLED_PROBE_STEP +
                             (nb + SAMPLED_PROBE_STEP - 1) / SAMPLED_PROBE_STEP;
    TJ_CK(x.timed(F_PROBE, sampled * (uint64_t)x.sh.kb, [&] {
        return launch_probe_step(x.sh.kb, a, na, b, nb, SAMPLED_PROBE_STEP, x.d_probe, x.st);
    }));
    TJ_CK(hipMemcpyAsync(mm, x.d_probe, 16, hipMemcpyDeviceToHost, x.st));
    TJ_CK(hipStreamSynchronize(x.st));
    x.stats.bytes_read += sampled * (uint64_t)x.sh.kb;
    hi = mm[1];
    lo = mm[0];
    // the digit width depends on the span, which depends on the rounded minimum
    for (int it = 0; it < 3; it++) {
        uint32_t shift, bits;
        plan_digit(hi - lo, na + nb, true, shift, bits);  // as the first pass (one segment)
        const uint64_t aligned = shift >= 64 ? 0 : (mm[0] & ~((1ull << shift) - 1));
        if (aligned == lo) break;
        lo = aligned;
    }
    return TJ_OK;
}

// TJ_PART_AUTO on a call with a sampled first range: the digit histogram of
// that sample (every SAMPLED_PROBE_STEP-th key of each side, gathered into
// `scratch`, device memory nothing uses yet) takes the decision the first
// pass's histogram would take, without a pass over the rows: learned when one
// bucket of the first radix digit over [lo, hi] holds more than half of them.
int sample_wants_learned(Exec& x, const void* a, uint64_t na, const void* b, uint64_t nb, uint64_t lo,
                         uint64_t hi, uint64_t* scratch, bool& learned)
{
    const uint64_t ma = (na + SAMPLED_PROBE_STEP - 1) / SAMPLED_PROBE_STEP;
    const uint64_t mb = (nb + SAMPLED_PROBE_STEP - 1) / SAMPLED_PROBE_STEP;
    TJ_CK(launch_gather_step(x.sh.kb, a, na, SAMPLED_PROBE_STEP, scratch, x.st));
    if (nb) TJ_CK(launch_gather_step(x.sh.kb, b, nb, SAMPLED_PROBE_STEP, scratch + ma, x.st));
    uint64_t* h = (uint64_t*)pinned_down((size_t)(ma + mb) * 8);
    if (!h) return TJ_E_HIP;
    TJ_CK(hipMemcpyAsync(h, scratch, (size_t)(ma + mb) * 8, hipMemcpyDeviceToHost, x.st));
    TJ_CK(hipStreamSynchronize(x.st));
    x.stats.bytes_read += (ma + mb) * (uint64_t)x.sh.kb;
    uint32_t shift, bits;
    plan_digit(hi - lo, na + nb, true, shift, bits);  // the first pass's digit
    std::vector<uint64_t> cnt((size_t)1 << bits, 0);
    const uint64_t mask = (1ull << bits) - 1;
    uint64_t largest = 0;
    for (uint64_t i = 0; i < ma + mb; i++) {
        const uint64_t o = h[i];
        if (o < lo || o > hi) continue;
        const uint64_t c = ++cnt[(size_t)(((o - lo) >> shift) & mask)];
        largest = std::max(largest, c);
    }
    learned = AUTO_BULK_DEN * largest > ma + mb;
    return TJ_OK;
}

}  // namespace
}  // namespace tj

using namespace tj;

extern "C" {

const char* tj_strerror(int status)
{
    switch (status) {
    case TJ_OK: return "ok";
    case TJ_E_ARG: return "invalid argument";
    case TJ_E_WORKSPACE: return "workspace too small or misaligned";
    case TJ_E_CAPACITY: return "join result exceeds output capacity";
    case TJ_E_TOO_LARGE: return "row count must be below 2^31";
    case TJ_E_ALIAS: return "output overlaps an input or the workspace";
    case TJ_E_HIP: return "HIP runtime error";
    case TJ_E_INTERNAL: return "internal planner error";
    default: return "unknown status";
    }
}

int tj_version(void) { return 100; }

int tj_timing(int enable)
{
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    if (enable && !t.on) {
        for (int f = 0; f < NFAM; f++) {
            t.launches[f] = 0;
            t.bytes[f] = 0;
            t.ms[f] = 0;
        }
    }
    t.on = enable != 0;
    return TJ_OK;
}

int tj_timing_read(tj_kernel_stat_t* out, int max)
{
    if (!out || max < 0) return TJ_E_ARG;
    Timing& t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    int n = 0;
    for (int f = 0; f < NFAM && n < max; f++, n++) {
        std::memset(&out[n], 0, sizeof(out[n]));
        std::strncpy(out[n].name, kFamName[f], sizeof(out[n].name) - 1);
        out[n].launches = t.launches[f];
        out[n].bytes = t.bytes[f];
        out[n].ms = t.ms[f];
    }
    return n;
}

int tj_workspace_query(int op, int key_type, uint64_t n_r, uint64_t n_s, uint64_t* min_bytes,
                       uint64_t* full_bytes)
{
    if (validate_common(key_type) != TJ_OK) return TJ_E_ARG;
    if (op != TJ_OP_SORT && op != TJ_OP_JOIN_COUNT && op != TJ_OP_JOIN_MATERIALIZE) return TJ_E_ARG;
    if (!min_bytes || !full_bytes) return TJ_E_ARG;
    if (n_r > kMaxRows || (op != TJ_OP_SORT && n_s > kMaxRows)) return TJ_E_TOO_LARGE;
    Shape s{op, key_type, op != TJ_OP_SORT, op == TJ_OP_JOIN_MATERIALIZE, op != TJ_OP_JOIN_COUNT,
            n_r, op == TJ_OP_SORT ? 0 : n_s};
    *min_bytes = min_workspace(s);
    *full_bytes = full_workspace(s);
    return TJ_OK;
}

}  // extern "C"

namespace tj {
namespace {

// Learned options in effect for a call: false means the radix path.
int learned_wanted(const tj_options_t* opt, uint64_t rows, bool& want, bool& is_auto, uint32_t& permille)
{
    want = false;
    is_auto = opt && opt->partitioner == TJ_PART_AUTO;
    permille = DEFAULT_PERMILLE;
    if (!opt) return TJ_OK;
    if (opt->partitioner != TJ_PART_RADIX && opt->partitioner != TJ_PART_LEARNED &&
        opt->partitioner != TJ_PART_AUTO)
        return TJ_E_ARG;
    if (opt->partitioner == TJ_PART_RADIX) return TJ_OK;
    if (opt->sample_permille > 1000) return TJ_E_ARG;
    if (opt->sample_permille) permille = opt->sample_permille;
    uint64_t min_rows = opt->learned_min_rows ? opt->learned_min_rows : DEFAULT_LEARNED_MIN_ROWS;
    if (min_rows < (uint64_t)LEAF_CAP + 1) min_rows = (uint64_t)LEAF_CAP + 1;
    want = rows >= min_rows;
    return TJ_OK;
}

}  // namespace
}  // namespace tj

static int sort_body(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n, void* keys_out,
                     int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream,
                     const tj_options_t* opt, tj_stats_t* stats)
{
    if (validate_common(key_type) != TJ_OK) return TJ_E_ARG;
    bool want_learned, is_auto;
    uint32_t permille;
    TJ_RET(learned_wanted(opt, n, want_learned, is_auto, permille));
    if (n > kMaxRows) return TJ_E_TOO_LARGE;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0) return TJ_OK;
    if (!keys_in || !rids_in || !keys_out || !rids_out || !workspace) return TJ_E_ARG;
    if ((uintptr_t)workspace % ALIGN) return TJ_E_WORKSPACE;
    const uint64_t kbytes = n * (uint64_t)key_type, rbytes = n * 4;
    const void* outs[2] = {keys_out, rids_out};
    const uint64_t osz[2] = {kbytes, rbytes};
    for (int i = 0; i < 2; i++)
        if (overlap(outs[i], osz[i], keys_in, kbytes) || overlap(outs[i], osz[i], rids_in, rbytes) ||
            overlap(outs[i], osz[i], workspace, workspace_bytes))
            return TJ_E_ALIAS;
    if (overlap(keys_out, kbytes, rids_out, rbytes)) return TJ_E_ALIAS;
    if (overlap(workspace, workspace_bytes, keys_in, kbytes) || overlap(workspace, workspace_bytes, rids_in, rbytes))
        return TJ_E_ALIAS;

    Exec x;
    x.timed_on = timing_enabled() && !t_nested && !t_noalloc;
    x.sh = Shape{TJ_OP_SORT, key_type, false, false, true, n, 0};
    x.st = (hipStream_t)stream;
    int tier;
    bool unlimited;
    uint64_t data_bytes;
    TJ_RET(plan_workspace(x.sh, workspace_bytes, tier, unlimited, data_bytes));
    x.caps = tier_caps(tier);
    char* p = (char*)workspace;
    char* end = p + workspace_bytes;
    TJ_RET(x.carve_tables(p, end));
    layout_data(x, p, data_bytes, unlimited, key_type);
    x.bufs.key[BUF_IN][0] = keys_in;
    x.bufs.rid[BUF_IN][0] = rids_in;
    x.bufs.key[BUF_A][0] = keys_out;
    x.bufs.rid[BUF_A][0] = rids_out;
    x.out_is_a = true;  // buffer A is the output (the budget plan's key ranges change that)

    // buffer B (workspace) is free until the second pass: the training
    // scratch, then the learned pass's bucket ids
    auto train = [&]() -> int {
        char* b0 = (char*)x.bufs.key[BUF_B][0];
        x.d_model = (tj_rmi_t*)b0;
        char* s0 = b0 + rmi_model_bytes();
        const int rc = x.train_rmi(keys_in, n, nullptr, 0, permille, s0, (uint64_t)(end - s0));
        if (rc == TJ_OK) {
            x.bkt.b[0] = (uint16_t*)s0;
            x.learned_pass = true;
            x.stats.learned = 1;
        }
        return rc;
    };
    bool learned = false;
    if (unlimited && want_learned && !is_auto) {
        const int rc = train();
        if (rc != TJ_OK && rc != TJ_E_WORKSPACE) return rc;
        learned = rc == TJ_OK;
    }
    uint64_t lo = 0, hi = ~0ull;
    bool spec = false;
    if (!learned) {
        // large unlimited calls take their first digit range from a sample (a
        // sampled span of 0 could hide other keys: probe those exactly)
        if (unlimited && n >= SAMPLED_PROBE_MIN_ROWS) {
            TJ_RET(sampled_range(x, keys_in, n, nullptr, 0, lo, hi));
            spec = hi > lo;
            if (spec && want_learned && is_auto) {
                // auto decides from the same sample (buffer B is still free)
                bool to_learned = false;
                TJ_RET(sample_wants_learned(x, keys_in, n, nullptr, 0, lo, hi, (uint64_t*)x.bufs.key[BUF_B][0],
                                            to_learned));
                is_auto = false;
                want_learned = to_learned;
                if (to_learned) {
                    const int rc = train();
                    if (rc != TJ_OK && rc != TJ_E_WORKSPACE) return rc;
                    learned = rc == TJ_OK;
                }
            }
        }
        if (!spec && !learned) TJ_RET(probe(x, keys_in, n, nullptr, 0, lo, hi));
    }
    if (unlimited) {
        x.stats.key_ranges = 1;
        x.auto_probe = want_learned && is_auto;
        x.spec_range = spec;
        int rc = learned ? x.process_range(0, ~0ull, n, 0, false, 0) : x.process_range(lo, hi, n, 0, false, 0);
        if (rc == TJ_RANGE_MISS) {
            TJ_RET(probe(x, keys_in, n, nullptr, 0, lo, hi));
            spec = false;
            rc = x.process_range(lo, hi, n, 0, false, 0);
        }
        if (rc == TJ_SWITCH_LEARNED) {
            const int tr = train();
            if (tr != TJ_OK && tr != TJ_E_WORKSPACE) return tr;
            x.auto_probe = false;
            x.spec_range = spec;  // still checked if the range is the sampled one
            rc = tr == TJ_OK ? x.process_range(0, ~0ull, n, 0, false, 0) : x.process_range(lo, hi, n, 0, false, 0);
        }
        TJ_RET(rc);
        TJ_RET(x.run_sort_leaves(keys_out, rids_out));
    } else {
        // the budget binds: output columns plus a workspace window (sort_windowed)
        x.stats.key_ranges = 1;
        TJ_RET(x.sort_windowed(lo, hi, n, 0, false, 0, keys_out, rids_out, (char*)x.bufs.key[BUF_B][0],
                               (char*)x.bufs.rid[BUF_B][0], x.cap_r));
    }
    TJ_CK(hipStreamSynchronize(x.st));
    x.stats.workspace_used = workspace_bytes;
    if (stats) *stats = x.stats;
    return TJ_OK;
}

static int join_body(int key_type, const void* r_keys, const int32_t* r_rids, uint64_t n_r,
                     const void* s_keys, const int32_t* s_rids, uint64_t n_s, int32_t* out_r,
                     int32_t* out_s, uint64_t capacity, uint64_t* count, void* workspace,
                     uint64_t workspace_bytes, void* stream, tj_stats_t* stats, bool mat,
                     const tj_options_t* opt)
{
    if (validate_common(key_type) != TJ_OK) return TJ_E_ARG;
    bool want_learned, is_auto;
    uint32_t permille;
    TJ_RET(learned_wanted(opt, n_r + n_s, want_learned, is_auto, permille));
    if (!count) return TJ_E_ARG;
    if (n_r > kMaxRows || n_s > kMaxRows) return TJ_E_TOO_LARGE;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    *count = 0;
    if (n_r == 0 || n_s == 0) return TJ_OK;
    if (!r_keys || !s_keys || !workspace) return TJ_E_ARG;
    if (mat && (!r_rids || !s_rids || (capacity > 0 && (!out_r || !out_s)))) return TJ_E_ARG;
    if ((uintptr_t)workspace % ALIGN) return TJ_E_WORKSPACE;
    const uint64_t kb = (uint64_t)key_type;
    if (overlap(workspace, workspace_bytes, r_keys, n_r * kb) || overlap(workspace, workspace_bytes, s_keys, n_s * kb) ||
        (mat && (overlap(workspace, workspace_bytes, r_rids, n_r * 4) ||
                 overlap(workspace, workspace_bytes, s_rids, n_s * 4))))
        return TJ_E_ALIAS;
    if (mat && capacity > 0) {
        const void* ins[4] = {r_keys, s_keys, r_rids, s_rids};
        const uint64_t isz[4] = {n_r * kb, n_s * kb, n_r * 4, n_s * 4};
        const void* outs[2] = {out_r, out_s};
        for (int o = 0; o < 2; o++) {
            for (int i = 0; i < 4; i++)
                if (overlap(outs[o], capacity * 4, ins[i], isz[i])) return TJ_E_ALIAS;
            if (overlap(outs[o], capacity * 4, workspace, workspace_bytes)) return TJ_E_ALIAS;
        }
        if (overlap(out_r, capacity * 4, out_s, capacity * 4)) return TJ_E_ALIAS;
    }

    Exec x;
    x.timed_on = timing_enabled() && !t_nested && !t_noalloc;
    x.sh = Shape{mat ? TJ_OP_JOIN_MATERIALIZE : TJ_OP_JOIN_COUNT, key_type, true, mat, mat, n_r, n_s};
    x.st = (hipStream_t)stream;
    int tier;
    bool unlimited;
    uint64_t data_bytes;
    TJ_RET(plan_workspace(x.sh, workspace_bytes, tier, unlimited, data_bytes));
    x.caps = tier_caps(tier);
    char* p = (char*)workspace;
    char* end = p + workspace_bytes;
    TJ_RET(x.carve_tables(p, end));
    layout_data(x, p, data_bytes, unlimited, key_type);
    x.bufs.key[BUF_IN][0] = r_keys;
    x.bufs.key[BUF_IN][1] = s_keys;
    x.bufs.rid[BUF_IN][0] = r_rids;
    x.bufs.rid[BUF_IN][1] = s_rids;

    // buffer B is free until the second pass (see tj_sort)
    auto train = [&]() -> int {
        char* b0 = (char*)x.bufs.key[BUF_B][0];
        x.d_model = (tj_rmi_t*)b0;
        char* s0 = b0 + rmi_model_bytes();
        const int rc = x.train_rmi(r_keys, n_r, s_keys, n_s, permille, s0, (uint64_t)(end - s0));
        if (rc == TJ_OK) {
            x.bkt.b[0] = (uint16_t*)s0;
            x.bkt.b[1] = (uint16_t*)(s0 + align_up(n_r * 2, ALIGN));
            x.learned_pass = true;
            x.stats.learned = 1;
        }
        return rc;
    };
    bool learned = false;
    if (unlimited && want_learned && !is_auto) {
        const int rc = train();
        if (rc != TJ_OK && rc != TJ_E_WORKSPACE) return rc;
        learned = rc == TJ_OK;
    }
    uint64_t lo = 0, hi = ~0ull;
    bool spec = false;
    if (!learned) {
        if (unlimited && n_r + n_s >= SAMPLED_PROBE_MIN_ROWS) {  // as in tj_sort
            TJ_RET(sampled_range(x, r_keys, n_r, s_keys, n_s, lo, hi));
            spec = hi > lo;
            if (spec && want_learned && is_auto) {
                bool to_learned = false;
                TJ_RET(sample_wants_learned(x, r_keys, n_r, s_keys, n_s, lo, hi, (uint64_t*)x.bufs.key[BUF_B][0],
                                            to_learned));
                is_auto = false;
                want_learned = to_learned;
                if (to_learned) {
                    const int rc = train();
                    if (rc != TJ_OK && rc != TJ_E_WORKSPACE) return rc;
                    learned = rc == TJ_OK;
                }
            }
        }
        if (!spec && !learned) TJ_RET(probe(x, r_keys, n_r, s_keys, n_s, lo, hi));
    }
    uint64_t total = 0;
    if (unlimited) {
        x.stats.key_ranges = 1;
        x.auto_probe = want_learned && is_auto;
        x.spec_range = spec;
        int rc = learned ? x.process_range(0, ~0ull, n_r, n_s, false, 0) : x.process_range(lo, hi, n_r, n_s, false, 0);
        if (rc == TJ_RANGE_MISS) {
            TJ_RET(probe(x, r_keys, n_r, s_keys, n_s, lo, hi));
            spec = false;
            rc = x.process_range(lo, hi, n_r, n_s, false, 0);
        }
        if (rc == TJ_SWITCH_LEARNED) {
            const int tr = train();
            if (tr != TJ_OK && tr != TJ_E_WORKSPACE) return tr;
            x.auto_probe = false;
            x.spec_range = spec;  // still checked if the range is the sampled one
            rc = tr == TJ_OK ? x.process_range(0, ~0ull, n_r, n_s, false, 0)
                             : x.process_range(lo, hi, n_r, n_s, false, 0);
        }
        TJ_RET(rc);
        TJ_RET(x.finish_join(&total, 0, out_r, out_s, capacity, mat));
    } else {
        // Ranges in key order; each range is counted, then written at the
        // running offset while the running total still fits the capacity.
        // When the whole key span is below 2^41, every range's filtered pass
        // narrows its keys to 4 bytes (a full digit leaves at most 2^32
        // ordinals per child), so the buffers hold 4-byte keys and more rows.
        // Those buffers are then also laid out unequally: most of the region
        // holds a range's rows, the rest is a window for its buckets that need
        // further passes (layout_join_window).
        if (key_type == 8 && hi - lo < (1ull << 41)) {
            x.narrow_ranges = true;
            layout_join_window(x, p, data_bytes);
        }
        std::vector<Exec::Range> ranges;
        TJ_RET(x.plan_ranges(lo, hi, ranges, 0));
        x.stats.key_ranges = (uint32_t)ranges.size();
        for (const auto& r : ranges) {
            if (r.rn == 0 || r.sn == 0) continue;
            if (r.lo == r.hi) {
                if (mat && total + r.rn * r.sn <= capacity)
                    TJ_RET(x.single_key_pairs(r.lo, r.rn, r.sn, total, out_r, out_s));
                total += r.rn * r.sn;
                continue;
            }
            if (r.rn > x.cap_r || r.sn > x.cap_s) return TJ_E_INTERNAL;
            uint64_t t = 0;
            TJ_RET(x.process_range(r.lo, r.hi, r.rn, r.sn, true, 0));
            TJ_RET(x.finish_join(&t, total, out_r, out_s, capacity, mat));
            total += t;
        }
    }
    *count = total;
    TJ_CK(hipStreamSynchronize(x.st));
    x.stats.workspace_used = workspace_bytes;
    if (stats) *stats = x.stats;
    if (mat && total > capacity) return TJ_E_CAPACITY;
    return TJ_OK;
}

// Host-side containers of the planner may throw (std::bad_alloc); nothing
// crosses the C ABI: an exception becomes TJ_E_INTERNAL.
static int sort_impl(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n, void* keys_out,
                     int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream,
                     const tj_options_t* opt, tj_stats_t* stats)
{
    try {
        return sort_body(key_type, keys_in, rids_in, n, keys_out, rids_out, workspace, workspace_bytes, stream, opt,
                         stats);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

static int join_impl(int key_type, const void* r_keys, const int32_t* r_rids, uint64_t n_r,
                     const void* s_keys, const int32_t* s_rids, uint64_t n_s, int32_t* out_r,
                     int32_t* out_s, uint64_t capacity, uint64_t* count, void* workspace,
                     uint64_t workspace_bytes, void* stream, tj_stats_t* stats, bool mat,
                     const tj_options_t* opt)
{
    try {
        return join_body(key_type, r_keys, r_rids, n_r, s_keys, s_rids, n_s, out_r, out_s, capacity, count,
                         workspace, workspace_bytes, stream, stats, mat, opt);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

namespace tj {
// The sort of tj_sort with the workspace given by the caller of this
// function (the static scratch of tj_sort_static); no pinned staging and no
// timing events.
int sort_noalloc(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n, void* keys_out,
                 int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream, tj_stats_t* stats)
{
    struct Flag {
        bool saved = t_noalloc;
        Flag() { t_noalloc = true; }
        ~Flag() { t_noalloc = saved; }
    } flag;
    return sort_impl(key_type, keys_in, rids_in, n, keys_out, rids_out, workspace, workspace_bytes, stream,
                     nullptr, stats);
}

// Frees the calling thread's pinned staging and host lists. For a thread that
// made calls and is about to end (a server worker): it runs in ordinary code,
// not in a thread-exit destructor, and a later call on the same thread would
// simply allocate them again.
void release_thread_staging() { free_thread_staging(); }
}  // namespace tj

extern "C" {

int tj_sort(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n, void* keys_out,
            int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream,
            tj_stats_t* stats)
{
    return sort_impl(key_type, keys_in, rids_in, n, keys_out, rids_out, workspace, workspace_bytes, stream,
                     nullptr, stats);
}

int tj_sort_ex(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n, void* keys_out,
               int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream,
               const tj_options_t* opt, tj_stats_t* stats)
{
    return sort_impl(key_type, keys_in, rids_in, n, keys_out, rids_out, workspace, workspace_bytes, stream,
                     opt, stats);
}

int tj_join_count(int key_type, const void* r_keys, uint64_t n_r, const void* s_keys, uint64_t n_s,
                  uint64_t* count, void* workspace, uint64_t workspace_bytes, void* stream,
                  tj_stats_t* stats)
{
    return join_impl(key_type, r_keys, nullptr, n_r, s_keys, nullptr, n_s, nullptr, nullptr, 0, count,
                     workspace, workspace_bytes, stream, stats, false, nullptr);
}

int tj_join_count_ex(int key_type, const void* r_keys, uint64_t n_r, const void* s_keys, uint64_t n_s,
                     uint64_t* count, void* workspace, uint64_t workspace_bytes, void* stream,
                     const tj_options_t* opt, tj_stats_t* stats)
{
    return join_impl(key_type, r_keys, nullptr, n_r, s_keys, nullptr, n_s, nullptr, nullptr, 0, count,
                     workspace, workspace_bytes, stream, stats, false, opt);
}

int tj_join_materialize(int key_type, const void* r_keys, const int32_t* r_rids, uint64_t n_r,
                        const void* s_keys, const int32_t* s_rids, uint64_t n_s, int32_t* out_r,
                        int32_t* out_s, uint64_t capacity, uint64_t* count, void* workspace,
                        uint64_t workspace_bytes, void* stream, tj_stats_t* stats)
{
    return join_impl(key_type, r_keys, r_rids, n_r, s_keys, s_rids, n_s, out_r, out_s, capacity, count,
                     workspace, workspace_bytes, stream, stats, true, nullptr);
}

int tj_join_materialize_ex(int key_type, const void* r_keys, const int32_t* r_rids, uint64_t n_r,
                           const void* s_keys, const int32_t* s_rids, uint64_t n_s, int32_t* out_r,
                           int32_t* out_s, uint64_t capacity, uint64_t* count, void* workspace,
                           uint64_t workspace_bytes, void* stream, const tj_options_t* opt, tj_stats_t* stats)
{
    return join_impl(key_type, r_keys, r_rids, n_r, s_keys, s_rids, n_s, out_r, out_s, capacity, count,
                     workspace, workspace_bytes, stream, stats, true, opt);
}

int tj_rmi_workspace_query(int key_type, uint64_t n_a, uint64_t n_b, uint32_t permille, uint64_t* bytes)
{
    if (validate_common(key_type) != TJ_OK || !bytes || n_a == 0 || permille > 1000) return TJ_E_ARG;
    if (n_a > kMaxRows || n_b > kMaxRows) return TJ_E_TOO_LARGE;
    if (!permille) permille = DEFAULT_PERMILLE;
    const uint64_t M = rmi_sample_rows(n_a, permille) + (n_b ? rmi_sample_rows(n_b, permille) : 0);
    *bytes = align_up(sizeof(tj_rmi_t), ALIGN) + rmi_scratch_bytes(key_type, M, true);
    return TJ_OK;
}

}  // extern "C"

static int rmi_train_body(int key_type, const void* keys_a, uint64_t n_a, const void* keys_b, uint64_t n_b,
                 uint32_t permille, tj_rmi_t* model, void* workspace, uint64_t workspace_bytes, void* stream)
{
    if (validate_common(key_type) != TJ_OK || !keys_a || n_a == 0 || !model || !workspace) return TJ_E_ARG;
    if (n_b && !keys_b) return TJ_E_ARG;
    uint64_t need;
    TJ_RET(tj_rmi_workspace_query(key_type, n_a, n_b, permille, &need));
    if ((uintptr_t)workspace % ALIGN || workspace_bytes < need) return TJ_E_WORKSPACE;
    if (!permille) permille = DEFAULT_PERMILLE;
    Exec x;
    x.timed_on = timing_enabled() && !t_nested && !t_noalloc;
    x.sh = Shape{TJ_OP_SORT, key_type, false, false, true, n_a, n_b};
    x.st = (hipStream_t)stream;
    char* p = (char*)workspace;
    x.d_model = (tj_rmi_t*)p;
    p += align_up(sizeof(tj_rmi_t), ALIGN);
    TJ_RET(x.train_rmi(keys_a, n_a, keys_b, n_b, permille, p, (uint64_t)((char*)workspace + workspace_bytes - p)));
    TJ_CK(hipMemcpyAsync(model, x.d_model, sizeof(tj_rmi_t), hipMemcpyDeviceToHost, x.st));
    TJ_CK(hipStreamSynchronize(x.st));
    return TJ_OK;
}

extern "C" {

int tj_rmi_train(int key_type, const void* keys_a, uint64_t n_a, const void* keys_b, uint64_t n_b,
                 uint32_t permille, tj_rmi_t* model, void* workspace, uint64_t workspace_bytes, void* stream)
{
    try {
        return rmi_train_body(key_type, keys_a, n_a, keys_b, n_b, permille, model, workspace, workspace_bytes,
                              stream);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

int tj_rmi_buckets(int key_type, const void* keys, uint64_t n, const tj_rmi_t* model, uint16_t* buckets,
                   void* workspace, uint64_t workspace_bytes, void* stream)
{
    if (validate_common(key_type) != TJ_OK || !model) return TJ_E_ARG;
    if (n > kMaxRows) return TJ_E_TOO_LARGE;
    if (model->buckets == 0 || model->buckets > (uint32_t)NB) return TJ_E_ARG;
    for (int i = 0; i < TJ_RMI_SEGMENTS; i++)
        if (model->knot[i] > model->knot[i + 1] || !(model->knot_inv[i] >= 0.0f) || std::isinf(model->knot_inv[i]))
            return TJ_E_ARG;
    for (int l = 0; l < TJ_RMI_LEAVES; l++) {
        if (model->leaf_lo[l] > model->leaf_hi[l] || model->leaf_hi[l] >= model->buckets) return TJ_E_ARG;
        if (l + 1 < TJ_RMI_LEAVES && model->leaf_hi[l] > model->leaf_lo[l + 1]) return TJ_E_ARG;
        if (!std::isfinite(model->leaf_a[l]) || !(model->leaf_b[l] >= 0.0f) || std::isinf(model->leaf_b[l]))
            return TJ_E_ARG;
    }
    if (n == 0) return TJ_OK;
    if (!keys || !buckets || !workspace) return TJ_E_ARG;
    if ((uintptr_t)workspace % ALIGN || workspace_bytes < sizeof(tj_rmi_t)) return TJ_E_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    TJ_CK(hipMemcpyAsync(workspace, model, sizeof(tj_rmi_t), hipMemcpyHostToDevice, st));
    TJ_CK(launch_rmi_eval(key_type, keys, n, (const tj_rmi_t*)workspace, buckets, st));
    return TJ_OK;
}

}  // extern "C"

static int partition_pass_body(const int64_t* keys, const int32_t* rids, uint64_t n, uint64_t base,
                            uint32_t shift, uint32_t bits, uint32_t flags, int64_t* keys_out,
                            int32_t* rids_out, uint32_t* counts_out, void* workspace,
                            uint64_t workspace_bytes, void* stream)
{
    if (!keys || !rids || !keys_out || !rids_out || !counts_out || !workspace) return TJ_E_ARG;
    if (bits < 1 || bits > (uint32_t)MAX_DIGIT_BITS || shift > 63 || shift + bits > 64) return TJ_E_ARG;
    if (flags & ~(uint32_t)TJ_DEBUG_FORCE_REORDER) return TJ_E_ARG;
    if (n == 0 || n > kMaxRows) return n ? TJ_E_TOO_LARGE : TJ_E_ARG;
    if ((uintptr_t)workspace % ALIGN) return TJ_E_WORKSPACE;
    Exec x;
    x.sh = Shape{TJ_OP_SORT, 8, false, false, true, n, 0};
    x.st = (hipStream_t)stream;
    int tier = TABLE_TIERS - 1;
    while (tier > 0 && table_bytes(tier_caps(tier)) > workspace_bytes) tier--;
    x.caps = tier_caps(tier);
    char* p = (char*)workspace;
    TJ_RET(x.carve_tables(p, (char*)workspace + workspace_bytes));
    x.bufs.key[BUF_IN][0] = keys;
    x.bufs.rid[BUF_IN][0] = rids;
    x.bufs.key[BUF_A][0] = keys_out;
    x.bufs.rid[BUF_A][0] = rids_out;
    GroupDesc g{};
    g.len = n;
    g.base = base;
    g.flo = 0;
    g.fhi = ~0ull;
    g.shift = shift;
    g.bits = bits;
    g.src = BUF_IN;
    g.dst = BUF_A;
    g.flags = (flags & TJ_DEBUG_FORCE_REORDER) ? GROUP_FORCE_REORDER : 0u;
    std::vector<ChunkDesc> chunks;
    uint64_t ch = std::max<uint64_t>(PART_TILE, align_up((n + TARGET_CHUNKS - 1) / TARGET_CHUNKS, PART_TILE));
    while ((n + ch - 1) / ch > x.caps.chunks) ch *= 2;
    for (uint64_t c0 = 0; c0 < n; c0 += ch)
        chunks.push_back(ChunkDesc{c0, (uint32_t)std::min<uint64_t>(ch, n - c0), 0,
                                   (uint32_t)(chunks.size() / CBLOCK), 0});
    g.nchunks = (uint32_t)chunks.size();
    std::vector<CBlockDesc> cbs;
    for (uint32_t c = 0; c < g.nchunks; c += CBLOCK)
        cbs.push_back(CBlockDesc{0, c, std::min<uint32_t>(CBLOCK, g.nchunks - c), 0});
    g.ncblocks = (uint32_t)cbs.size();
    hipStream_t st = x.st;
    TJ_CK(hipMemcpyAsync(x.d_groups, &g, sizeof(g), hipMemcpyHostToDevice, st));
    TJ_CK(hipMemcpyAsync(x.d_chunks, chunks.data(), chunks.size() * sizeof(ChunkDesc), hipMemcpyHostToDevice, st));
    TJ_CK(hipMemcpyAsync(x.d_cblocks, cbs.data(), cbs.size() * sizeof(CBlockDesc), hipMemcpyHostToDevice, st));
    TJ_CK(launch_fill_u64(x.d_gmin, 1u << bits, ~0ull, st));
    TJ_CK(launch_fill_u64(x.d_gmax, 1u << bits, 0ull, st));
    TJ_CK(launch_hist(8, x.d_chunks, g.nchunks, x.d_groups, x.bufs, x.d_hist, x.d_gmin, x.d_gmax, nullptr, st));
    TJ_CK(launch_scan(x.d_cblocks, g.ncblocks, x.d_groups, 1, x.d_hist, x.d_cbsum, x.d_ccount, x.d_cstart, st));
    TJ_CK(launch_scatter(8, 8, true, true, x.d_chunks, g.nchunks, x.d_groups, x.d_hist, x.d_cbsum, x.d_cstart, x.bufs, st));
    TJ_CK(hipMemcpyAsync(counts_out, x.d_ccount, (1u << bits) * 4ull, hipMemcpyDeviceToDevice, st));
    TJ_CK(hipStreamSynchronize(st));
    return TJ_OK;
}

extern "C" {

int tj_debug_partition_pass(const int64_t* keys, const int32_t* rids, uint64_t n, uint64_t base,
                            uint32_t shift, uint32_t bits, uint32_t flags, int64_t* keys_out,
                            int32_t* rids_out, uint32_t* counts_out, void* workspace,
                            uint64_t workspace_bytes, void* stream)
{
    try {
        return partition_pass_body(keys, rids, n, base, shift, bits, flags, keys_out, rids_out, counts_out,
                                   workspace, workspace_bytes, stream);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

int tj_debug_set_flags(uint32_t flags)
{
    if (flags & ~(uint32_t)(TJ_DEBUG_FORCE_REORDER | TJ_DEBUG_FAIL_HOST_ALLOC)) return TJ_E_ARG;
    g_debug_flags.store(flags);
    return TJ_OK;
}

int tj_debug_stream_copy(const void* src, void* dst, uint64_t bytes, void* stream)
{
    if (!src || !dst || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16) return TJ_E_ARG;
    if (overlap(src, bytes, dst, bytes)) return TJ_E_ALIAS;
    return launch_stream_copy(src, dst, bytes, (hipStream_t)stream) == hipSuccess ? TJ_OK : TJ_E_HIP;
}

int tj_debug_wave_scan(const uint32_t* in, uint32_t* out, uint64_t n, void* stream)
{
    if (!in || !out || n % 64) return TJ_E_ARG;
    TJ_CK(launch_wave_scan_test(in, out, n, (hipStream_t)stream));
    TJ_CK(hipStreamSynchronize((hipStream_t)stream));
    return TJ_OK;
}

}  // extern "C"

// tj_multi.cpp - composite-key sort and join (tj_*_multi): key columns packed
// into one key when their bit widths allow, otherwise least-significant-group
// first stable sorts (sort) or a dense rank of the tuples (join), on top of
// the single-key calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "tj_internal.h"

using namespace tj;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kMaxRows = (1ull << 31) - 1;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline uint32_t nbits64(uint64_t x) { return x ? 64u - (uint32_t)__builtin_clzll(x) : 0u; }

#define MK_CK(expr)                                   \
    do {                                              \
        if ((expr) != hipSuccess) return TJ_E_HIP;    \
    } while (0)
#define MK_RET(expr)                                  \
    do {                                              \
        const int r_ = (expr);                        \
        if (r_ != TJ_OK) return r_;                   \
    } while (0)

bool overlap(const void* a, uint64_t an, const void* b, uint64_t bn)
{
    if (!a || !b || !an || !bn) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

// Bump allocator over the workspace.
struct Carve {
    char* p;
    char* end;
    char* take(uint64_t bytes)
    {
        char* q = p;
        p += align_up(bytes);
        return q;
    }
    bool ok() const { return p <= end; }
    uint64_t left() const { return p < end ? (uint64_t)(end - p) : 0; }
};

uint64_t ws_full(int op, int kt, uint64_t n_r, uint64_t n_s)
{
    uint64_t mn = 0, full = 0;
    tj_workspace_query(op, kt, n_r, n_s, &mn, &full);
    return full;
}

uint64_t ws_min(int op, int kt, uint64_t n_r, uint64_t n_s)
{
    uint64_t mn = 0, full = 0;
    tj_workspace_query(op, kt, n_r, n_s, &mn, &full);
    return mn;
}

int check_cols(int ncols, const int* types)
{
    if (ncols < 1 || ncols > TJ_MAX_KEY_COLS || !types) return TJ_E_ARG;
    for (int c = 0; c < ncols; c++)
        if (types[c] != TJ_KEY_I32 && types[c] != TJ_KEY_I64) return TJ_E_ARG;
    return TJ_OK;
}

void add_stats(tj_stats_t& a, const tj_stats_t& b)
{
    a.bytes_read += b.bytes_read;
    a.bytes_written += b.bytes_written;
    a.passes += b.passes;
    a.leaves += b.leaves;
    a.single_key += b.single_key;
    a.key_ranges = std::max(a.key_ranges, b.key_ranges);
}

// Per-column [min, max] ordinal over rows of a (and b), read back to the host.
int column_ranges(int ncols, const int* types, const void* const* a, uint64_t na, const void* const* b,
                  uint64_t nb, uint64_t* d_mm, hipStream_t st, uint64_t* lo, uint64_t* hi, tj_stats_t& stats)
{
    std::vector<uint64_t> mm(2 * ncols);
    for (int c = 0; c < ncols; c++) {
        MK_CK(launch_probe(types[c], a[c], na, b ? b[c] : nullptr, b ? nb : 0, d_mm + 2 * c, st));
        stats.bytes_read += (na + (b ? nb : 0)) * (uint64_t)types[c];
    }
    MK_CK(hipMemcpyAsync(mm.data(), d_mm, 16 * ncols, hipMemcpyDeviceToHost, st));
    MK_CK(hipStreamSynchronize(st));
    for (int c = 0; c < ncols; c++) {
        lo[c] = mm[2 * c];
        hi[c] = mm[2 * c + 1];
    }
    return TJ_OK;
}

// Groups of consecutive columns of at most 64 packed bits, least significant
// group first; a group's last column takes the low bits.
struct Group {
    int c0, c1;      // columns [c0, c1]
    uint32_t bits;   // packed width
};

std::vector<Group> plan_groups(int ncols, const uint32_t* bits)
{
    std::vector<Group> g;
    int c1 = ncols - 1;
    uint32_t acc = 0;
    for (int c = ncols - 1; c >= 0; c--) {
        if (acc + bits[c] > 64) {
            g.push_back(Group{c + 1, c1, acc});
            c1 = c;
            acc = 0;
        }
        acc += bits[c];
    }
    g.push_back(Group{0, c1, acc});
    return g;
}

PackArgs pack_args(const Group& g, const int* types, const void* const* a, const void* const* b, uint64_t na,
                   const uint64_t* lo, const uint32_t* bits)
{
    PackArgs p{};
    p.ncols = g.c1 - g.c0 + 1;
    p.n_a = na;
    uint32_t shift = 0;
    for (int c = g.c1; c >= g.c0; c--) {
        const int k = c - g.c0;
        p.col_a[k] = a[c];
        p.col_b[k] = b ? b[c] : a[c];
        p.kb[k] = types[c];
        p.min[k] = lo[c];
        p.shift[k] = bits[c] ? shift : 64u;
        shift += bits[c];
    }
    return p;
}

// Stable lexicographic order of the rows of a (and b, rows na..) by the key
// columns: `perm` (n rows, device) receives the sorted row indices. Scratch:
// perm2 (n int32), k0/k1 (n int64 each), inner workspace.
int order_rows(int ncols, const int* types, const void* const* a, const void* const* b, uint64_t na, uint64_t n,
               const uint64_t* lo, const uint32_t* bits, int32_t* perm, int32_t* perm2, void* k0, void* k1,
               char* inner, uint64_t inner_bytes, hipStream_t st, tj_stats_t& stats)
{
    const std::vector<Group> groups = plan_groups(ncols, bits);
    MK_CK(launch_iota(perm, n, st));
    int32_t* cur = perm;
    int32_t* nxt = perm2;
    for (size_t gi = 0; gi < groups.size(); gi++) {
        const Group& g = groups[gi];
        const int kb = g.bits <= 32 ? 4 : 8;
        const PackArgs pa = pack_args(g, types, a, b, na, lo, bits);
        // the first sort reads rows in input order; later ones in the current order
        MK_CK(launch_pack(pa, gi ? cur : nullptr, n, k0, kb, st));
        tj_stats_t s{};
        MK_RET(tj_sort(kb, k0, cur, n, k1, nxt, inner, inner_bytes, st, &s));
        add_stats(stats, s);
        std::swap(cur, nxt);
    }
    if (cur != perm) MK_CK(hipMemcpyAsync(perm, cur, n * 4, hipMemcpyDeviceToDevice, st));
    return TJ_OK;
}

uint64_t sort_fixed_bytes(uint64_t n)
{
    return align_up(16 * TJ_MAX_KEY_COLS) + 2 * align_up(n * 4) + 2 * align_up(n * 8);
}

int join_impl(int ncols, const int* types, const void* const* r_keys, const int32_t* r_rids, uint64_t n_r,
              const void* const* s_keys, const int32_t* s_rids, uint64_t n_s, int32_t* out_r, int32_t* out_s,
              uint64_t capacity, uint64_t* count, void* workspace, uint64_t ws_bytes, void* stream,
              tj_stats_t* stats, bool mat)
{
    MK_RET(check_cols(ncols, types));
    if (!count) return TJ_E_ARG;
    if (n_r > kMaxRows || n_s > kMaxRows || n_r + n_s > kMaxRows) return TJ_E_TOO_LARGE;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    *count = 0;
    if (n_r == 0 || n_s == 0) return TJ_OK;
    if (!r_keys || !s_keys || !workspace) return TJ_E_ARG;
    for (int c = 0; c < ncols; c++)
        if (!r_keys[c] || !s_keys[c]) return TJ_E_ARG;
    if (mat && (!r_rids || !s_rids || (capacity && (!out_r || !out_s)))) return TJ_E_ARG;
    if ((uintptr_t)workspace % kAlign) return TJ_E_WORKSPACE;
    for (int c = 0; c < ncols; c++)
        if (overlap(workspace, ws_bytes, r_keys[c], n_r * types[c]) ||
            overlap(workspace, ws_bytes, s_keys[c], n_s * types[c]))
            return TJ_E_ALIAS;
    if (mat && (overlap(workspace, ws_bytes, r_rids, n_r * 4) || overlap(workspace, ws_bytes, s_rids, n_s * 4)))
        return TJ_E_ALIAS;
    if (mat && capacity) {
        for (int c = 0; c < ncols; c++)
            for (int32_t* o : {out_r, out_s})
                if (overlap(o, capacity * 4, r_keys[c], n_r * types[c]) ||
                    overlap(o, capacity * 4, s_keys[c], n_s * types[c]))
                    return TJ_E_ALIAS;
        for (int32_t* o : {out_r, out_s})
            if (overlap(o, capacity * 4, r_rids, n_r * 4) || overlap(o, capacity * 4, s_rids, n_s * 4) ||
                overlap(o, capacity * 4, workspace, ws_bytes))
                return TJ_E_ALIAS;
        if (overlap(out_r, capacity * 4, out_s, capacity * 4)) return TJ_E_ALIAS;
    }
    hipStream_t st = (hipStream_t)stream;
    tj_stats_t acc{};
    Carve cv{(char*)workspace, (char*)workspace + ws_bytes};
    uint64_t* d_mm = (uint64_t*)cv.take(16 * TJ_MAX_KEY_COLS);
    if (!cv.ok()) return TJ_E_WORKSPACE;
    uint64_t lo[TJ_MAX_KEY_COLS], hi[TJ_MAX_KEY_COLS];
    uint32_t bits[TJ_MAX_KEY_COLS];
    MK_RET(column_ranges(ncols, types, r_keys, n_r, s_keys, n_s, d_mm, st, lo, hi, acc));
    uint32_t total = 0;
    for (int c = 0; c < ncols; c++) {
        bits[c] = lo[c] <= hi[c] ? nbits64(hi[c] - lo[c]) : 0;
        total += bits[c];
    }
    const uint64_t N = n_r + n_s;
    void *kr, *ks;
    int kt;
    if (total <= 64) {
        // one packed key per row
        kt = total <= 32 ? 4 : 8;
        kr = cv.take(n_r * kt);
        ks = cv.take(n_s * kt);
        if (!cv.ok()) return TJ_E_WORKSPACE;
        const Group g{0, ncols - 1, total};
        const PackArgs pr = pack_args(g, types, r_keys, nullptr, n_r, lo, bits);
        const PackArgs ps = pack_args(g, types, s_keys, nullptr, n_s, lo, bits);
        MK_CK(launch_pack(pr, nullptr, n_r, kr, kt, st));
        MK_CK(launch_pack(ps, nullptr, n_s, ks, kt, st));
    } else {
        // dense rank of the tuples over R and S together, in tuple order
        kt = 4;
        int32_t* rank = (int32_t*)cv.take(N * 4);
        Carve sc = cv;  // scratch, dead once the ranks are written
        int32_t* perm = (int32_t*)sc.take(N * 4);
        int32_t* perm2 = (int32_t*)sc.take(N * 4);
        void* k0 = sc.take(N * 8);
        void* k1 = sc.take(N * 8);
        uint32_t* flag = (uint32_t*)sc.take(N * 4);
        uint32_t* dense = (uint32_t*)sc.take(N * 4);
        uint32_t* scan_tmp = (uint32_t*)sc.take(scan_scratch_words(N) * 4);
        if (!sc.ok() || sc.left() < ws_min(TJ_OP_SORT, 8, N, 0)) return TJ_E_WORKSPACE;
        MK_RET(order_rows(ncols, types, r_keys, s_keys, n_r, N, lo, bits, perm, perm2, k0, k1, sc.p, sc.left(), st,
                          acc));
        PackArgs pa = pack_args(Group{0, ncols - 1, total}, types, r_keys, s_keys, n_r, lo, bits);
        MK_CK(launch_tuple_flags(pa, perm, N, flag, st));
        MK_CK(launch_incl_scan(flag, N, scan_tmp, dense, st));
        MK_CK(launch_scatter_back(dense, perm, N, rank, st));
        acc.bytes_read += N * 16;
        acc.bytes_written += N * 12;
        kr = rank;
        ks = rank + n_r;
    }
    tj_stats_t s{};
    const int rc = mat ? tj_join_materialize(kt, kr, r_rids, n_r, ks, s_rids, n_s, out_r, out_s, capacity, count,
                                             cv.p, cv.left(), stream, &s)
                       : tj_join_count(kt, kr, n_r, ks, n_s, count, cv.p, cv.left(), stream, &s);
    add_stats(acc, s);
    acc.workspace_used = ws_bytes;
    if (stats) *stats = acc;
    return rc;
}

}  // namespace

extern "C" {

int tj_multi_workspace_query(int op, int ncols, const int* key_types, uint64_t n_r, uint64_t n_s, uint64_t* bytes)
{
    if (check_cols(ncols, key_types) != TJ_OK || !bytes) return TJ_E_ARG;
    if (op != TJ_OP_SORT && op != TJ_OP_JOIN_COUNT && op != TJ_OP_JOIN_MATERIALIZE) return TJ_E_ARG;
    if (n_r > kMaxRows || (op != TJ_OP_SORT && (n_s > kMaxRows || n_r + n_s > kMaxRows))) return TJ_E_TOO_LARGE;
    if (op == TJ_OP_SORT) {
        *bytes = sort_fixed_bytes(n_r) + ws_full(TJ_OP_SORT, 8, n_r, 0);
        return TJ_OK;
    }
    const uint64_t N = n_r + n_s;
    const uint64_t head = align_up(16 * TJ_MAX_KEY_COLS);
    const uint64_t packed = align_up(n_r * 8) + align_up(n_s * 8) + ws_full(op, 8, n_r, n_s);
    const uint64_t ranked = align_up(N * 4) +
                            std::max<uint64_t>(2 * align_up(N * 4) + 2 * align_up(N * 8) + 2 * align_up(N * 4) +
                                                   align_up(scan_scratch_words(N) * 4) + ws_full(TJ_OP_SORT, 8, N, 0),
                                               ws_full(op, 4, n_r, n_s));
    *bytes = head + std::max(packed, ranked);
    return TJ_OK;
}

static int sort_multi_body(int ncols, const int* key_types, const void* const* keys_in, const int32_t* rids_in,
                           uint64_t n, void* const* keys_out, int32_t* rids_out, void* workspace,
                           uint64_t workspace_bytes, void* stream, tj_stats_t* stats)
{
    MK_RET(check_cols(ncols, key_types));
    if (n > kMaxRows) return TJ_E_TOO_LARGE;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    if (n == 0) return TJ_OK;
    if (!keys_in || !rids_in || !keys_out || !rids_out || !workspace) return TJ_E_ARG;
    for (int c = 0; c < ncols; c++)
        if (!keys_in[c] || !keys_out[c]) return TJ_E_ARG;
    if ((uintptr_t)workspace % kAlign) return TJ_E_WORKSPACE;
    // outputs against inputs, the workspace and each other
    std::vector<std::pair<const void*, uint64_t>> ins, outs;
    for (int c = 0; c < ncols; c++) {
        ins.push_back({keys_in[c], n * key_types[c]});
        outs.push_back({keys_out[c], n * key_types[c]});
    }
    ins.push_back({rids_in, n * 4});
    ins.push_back({workspace, workspace_bytes});
    outs.push_back({rids_out, n * 4});
    for (size_t o = 0; o < outs.size(); o++) {
        for (auto& i : ins)
            if (overlap(outs[o].first, outs[o].second, i.first, i.second)) return TJ_E_ALIAS;
        for (size_t q = o + 1; q < outs.size(); q++)
            if (overlap(outs[o].first, outs[o].second, outs[q].first, outs[q].second)) return TJ_E_ALIAS;
    }
    for (size_t i = 0; i + 1 < ins.size(); i++)  // the workspace (last) against every input
        if (overlap(workspace, workspace_bytes, ins[i].first, ins[i].second)) return TJ_E_ALIAS;
    hipStream_t st = (hipStream_t)stream;
    tj_stats_t acc{};
    Carve cv{(char*)workspace, (char*)workspace + workspace_bytes};
    uint64_t* d_mm = (uint64_t*)cv.take(16 * TJ_MAX_KEY_COLS);
    int32_t* perm = (int32_t*)cv.take(n * 4);
    int32_t* perm2 = (int32_t*)cv.take(n * 4);
    void* k0 = cv.take(n * 8);
    void* k1 = cv.take(n * 8);
    if (!cv.ok() || cv.left() < ws_min(TJ_OP_SORT, 8, n, 0)) return TJ_E_WORKSPACE;
    uint64_t lo[TJ_MAX_KEY_COLS], hi[TJ_MAX_KEY_COLS];
    uint32_t bits[TJ_MAX_KEY_COLS];
    MK_RET(column_ranges(ncols, key_types, keys_in, n, nullptr, 0, d_mm, st, lo, hi, acc));
    for (int c = 0; c < ncols; c++) bits[c] = nbits64(hi[c] - lo[c]);
    MK_RET(order_rows(ncols, key_types, keys_in, nullptr, n, n, lo, bits, perm, perm2, k0, k1, cv.p, cv.left(), st,
                      acc));
    for (int c = 0; c < ncols; c++) MK_CK(launch_gather(key_types[c], keys_in[c], perm, n, keys_out[c], st));
    MK_CK(launch_gather(4, rids_in, perm, n, rids_out, st));
    for (int c = 0; c < ncols; c++) {
        acc.bytes_read += n * (uint64_t)key_types[c] + n * 4;
        acc.bytes_written += n * (uint64_t)key_types[c];
    }
    acc.bytes_read += n * 8;
    acc.bytes_written += n * 4;
    MK_CK(hipStreamSynchronize(st));
    acc.workspace_used = workspace_bytes;
    if (stats) *stats = acc;
    return TJ_OK;
}

int tj_sort_multi(int ncols, const int* key_types, const void* const* keys_in, const int32_t* rids_in, uint64_t n,
                  void* const* keys_out, int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream,
                  tj_stats_t* stats)
{
    try {  // host-side containers may throw; nothing crosses the C ABI
        return sort_multi_body(ncols, key_types, keys_in, rids_in, n, keys_out, rids_out, workspace, workspace_bytes,
                               stream, stats);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

int tj_join_count_multi(int ncols, const int* key_types, const void* const* r_keys, uint64_t n_r,
                        const void* const* s_keys, uint64_t n_s, uint64_t* count, void* workspace,
                        uint64_t workspace_bytes, void* stream, tj_stats_t* stats)
{
    try {
        return join_impl(ncols, key_types, r_keys, nullptr, n_r, s_keys, nullptr, n_s, nullptr, nullptr, 0, count,
                         workspace, workspace_bytes, stream, stats, false);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

int tj_join_materialize_multi(int ncols, const int* key_types, const void* const* r_keys, const int32_t* r_rids,
                              uint64_t n_r, const void* const* s_keys, const int32_t* s_rids, uint64_t n_s,
                              int32_t* out_r, int32_t* out_s, uint64_t capacity, uint64_t* count, void* workspace,
                              uint64_t workspace_bytes, void* stream, tj_stats_t* stats)
{
    try {
        return join_impl(ncols, key_types, r_keys, r_rids, n_r, s_keys, s_rids, n_s, out_r, out_s, capacity, count,
                         workspace, workspace_bytes, stream, stats, true);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

}  // extern "C"

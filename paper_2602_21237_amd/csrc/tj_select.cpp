// tj_select.cpp - execution-time path selection (tj_select_path): the
// indicators the paper names for the choice between the linear and the
// tensor path (input scale, join-key cardinality, expected intermediate size;
// Sec. III.C), observed on the device columns with a HyperLogLog sketch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "tj_internal.h"
#include "tj_select.h"

using namespace tj;

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint64_t kMaxRows = (1ull << 31) - 1;

inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool overlap(const void* a, uint64_t an, const void* b, uint64_t bn)
{
    if (!a || !b || !an || !bn) return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

struct Layout {
    uint64_t slab_r, slab_s, part, regs, whist, hist, total;
};

Layout layout(uint64_t n_r, uint64_t n_s)
{
    Layout l;
    l.slab_r = 0;
    l.slab_s = l.slab_r + align_up((uint64_t)hll_blocks(n_r) * HLL_M);
    l.part = l.slab_s + align_up((uint64_t)hll_blocks(n_s) * HLL_M);
    l.regs = l.part + align_up(2ull * HLL_GROUPS * HLL_M);
    l.whist = l.regs + align_up(3ull * HLL_M);
    l.hist = l.whist + align_up(HLL_WHIST_WORDS * sizeof(uint32_t));
    l.total = l.hist + align_up(3ull * HLL_BINS * sizeof(uint32_t));
    return l;
}

// The HyperLogLog estimate from the counts c[r] of registers holding rank r:
// raw estimate alpha_m m^2 / sum_j 2^-M[j], with the sum taken exactly as the
// integer sum_r c[r] 2^(51 - r); linear counting m ln(m / c[0]) below 2.5 m
// while some register is empty (Flajolet et al. 2007, Fig. 3).
double hll_estimate(const uint32_t* c)
{
    constexpr int kMaxRank = 64 - HLL_P + 1;
    unsigned __int128 z = 0;
    for (int r = 0; r <= kMaxRank; r++) z += (unsigned __int128)c[r] << (kMaxRank - r);
    const double m = (double)HLL_M;
    const double alpha = 0.7213 / (1.0 + 1.079 / m);
    const double am = alpha * m * m;
    double e = am * 0x1p51 / (double)z;
    if (e <= 2.5 * m && c[0] > 0) e = m * std::log(m / (double)c[0]);
    return e;
}

}  // namespace

extern "C" {

int tj_select_workspace_query(uint64_t n_r, uint64_t n_s, uint64_t* bytes)
{
    if (!bytes) return TJ_E_ARG;
    if (n_r > kMaxRows || n_s > kMaxRows) return TJ_E_TOO_LARGE;
    *bytes = layout(n_r, n_s).total;
    return TJ_OK;
}

int tj_select_path(int op, int key_type, const void* r_keys, uint64_t n_r, const void* s_keys, uint64_t n_s,
                   const tj_select_options_t* options, tj_selection_t* out, uint8_t* registers, void* workspace,
                   uint64_t workspace_bytes, void* stream)
{
    if (!out || (key_type != TJ_KEY_I32 && key_type != TJ_KEY_I64)) return TJ_E_ARG;
    if (op != TJ_OP_SORT && op != TJ_OP_JOIN_COUNT && op != TJ_OP_JOIN_MATERIALIZE) return TJ_E_ARG;
    const bool join = op != TJ_OP_SORT;
    if (!join && n_s != 0) return TJ_E_ARG;
    if ((n_r && !r_keys) || (join && n_s && !s_keys)) return TJ_E_ARG;
    if (n_r > kMaxRows || n_s > kMaxRows) return TJ_E_TOO_LARGE;
    const Layout l = layout(n_r, n_s);
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || workspace_bytes < l.total) return TJ_E_WORKSPACE;
    const uint64_t kb = (uint64_t)key_type;
    const uint64_t reg_bytes = 3ull * HLL_M;
    if (overlap(registers, reg_bytes, r_keys, n_r * kb) || overlap(registers, reg_bytes, s_keys, n_s * kb) ||
        overlap(registers, reg_bytes, workspace, workspace_bytes))
        return TJ_E_ALIAS;
    if (overlap(workspace, workspace_bytes, r_keys, n_r * kb) || overlap(workspace, workspace_bytes, s_keys, n_s * kb))
        return TJ_E_ALIAS;

    uint64_t min_rows = TJ_SELECT_DEFAULT_MIN_ROWS, min_output = TJ_SELECT_DEFAULT_MIN_OUTPUT;
    if (options) {
        if (options->min_rows) min_rows = options->min_rows;
        if (options->min_output) min_output = options->min_output;
    }

    hipStream_t st = (hipStream_t)stream;
    char* w = (char*)workspace;
    uint8_t* slab_r = (uint8_t*)(w + l.slab_r);
    uint8_t* slab_s = (uint8_t*)(w + l.slab_s);
    uint8_t* part = (uint8_t*)(w + l.part);
    uint8_t* regs = registers ? registers : (uint8_t*)(w + l.regs);
    uint32_t* d_whist = (uint32_t*)(w + l.whist);
    uint32_t* d_hist = (uint32_t*)(w + l.hist);
    if (launch_hll_block(key_type, r_keys, n_r, slab_r, st) != hipSuccess) return TJ_E_HIP;
    if (join && launch_hll_block(key_type, s_keys, n_s, slab_s, st) != hipSuccess) return TJ_E_HIP;
    const uint32_t nb_s = join ? hll_blocks(n_s) : 0;
    if (launch_hll_finish(slab_r, hll_blocks(n_r), slab_s, nb_s, part, regs, d_whist, d_hist, st) != hipSuccess)
        return TJ_E_HIP;
    uint32_t hist[3 * HLL_BINS];
    if (hipMemcpyAsync(hist, d_hist, sizeof(hist), hipMemcpyDeviceToHost, st) != hipSuccess) return TJ_E_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return TJ_E_HIP;

    tj_selection_t s{};
    s.n_r = n_r;
    s.n_s = join ? n_s : 0;
    s.distinct_r = hll_estimate(hist);
    s.distinct_s = join ? hll_estimate(hist + HLL_BINS) : 0.0;
    s.distinct_union = hll_estimate(hist + 2 * HLL_BINS);
    if (join) {
        const double common = s.distinct_r + s.distinct_s - s.distinct_union;
        s.distinct_common = std::max(0.0, std::min(std::min(s.distinct_r, s.distinct_s), common));
        if (s.distinct_r > 0 && s.distinct_s > 0)
            s.est_output = s.distinct_common * ((double)n_r / s.distinct_r) * ((double)n_s / s.distinct_s);
    }
    const uint64_t scale = n_r + s.n_s;
    s.reasons = (scale >= min_rows ? (uint32_t)TJ_SEL_SCALE : 0u) |
                (join && s.est_output >= (double)min_output ? (uint32_t)TJ_SEL_OUTPUT : 0u);
    s.path = s.reasons ? TJ_PATH_TENSOR : TJ_PATH_LINEAR;
    *out = s;
    return TJ_OK;
}

}  // extern "C"

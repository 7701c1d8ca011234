// tj_rmi.h - evaluation of the learned bucket function (two-layer RMI) on the
// device. The model layout and its definition are those of tj_rmi_t (tj.h);
// every float operation below is one IEEE f32 operation rounded to nearest
// even, and contraction into fused multiply-adds is switched off, so a model
// gives the same bucket on the device and in any other implementation that
// follows the definition.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "tj.h"

namespace tj {

constexpr uint64_t RMI_SAT = 1ull << 62;
constexpr uint32_t RMI_SUB = TJ_RMI_LEAVES / TJ_RMI_SEGMENTS;
static_assert(RMI_SUB == 4, "four leaves per root segment");
static_assert(sizeof(tj_rmi_t) % 16 == 0, "the model is copied in 16-byte words");

// Both layers are written without branches (selects, min/max), so that the
// evaluations of several rows interleave: each is a chain of dependent LDS
// reads.
__device__ __forceinline__ uint64_t rmi_min(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint64_t rmi_max(uint64_t a, uint64_t b) { return a > b ? a : b; }

// Root layer: the leaf of ordinal x. `m` may live in LDS or global memory.
__device__ __forceinline__ uint32_t rmi_leaf(const tj_rmi_t& m, uint64_t x)
{
#pragma clang fp contract(off)
    // largest j in [0, SEGMENTS - 1] with j == 0 or knot[j] <= x (knots non-decreasing)
    uint32_t j = 0;
#pragma unroll
    for (uint32_t step = TJ_RMI_SEGMENTS / 2; step >= 1; step >>= 1)
        j = m.knot[j + step] <= x ? j + step : j;
    const uint64_t lo = m.knot[j], hi = m.knot[j + 1];
    const uint64_t xc = rmi_min(rmi_max(x, lo), hi);
    const float t = (float)(xc - lo) * m.knot_inv[j];
    const float q = t * (float)RMI_SUB;  // exact: a power of two
    const uint32_t sub = q >= (float)(RMI_SUB - 1) ? RMI_SUB - 1 : (uint32_t)q;
    return j * RMI_SUB + sub;
}

// Leaf layer: the bucket of ordinal x, in [leaf_lo, leaf_hi] of its leaf.
__device__ __forceinline__ uint32_t rmi_bucket(const tj_rmi_t& m, uint64_t x)
{
#pragma clang fp contract(off)
    const uint32_t l = rmi_leaf(m, x);
    const uint64_t base = m.leaf_base[l];
    const bool ge = x >= base;
    const uint64_t dist = rmi_min(ge ? x - base : base - x, RMI_SAT);
    const int64_t sd = ge ? (int64_t)dist : -(int64_t)dist;
    const float prod = m.leaf_b[l] * (float)sd;
    const float y = m.leaf_a[l] + prod;
    const float lo = (float)m.leaf_lo[l], hi = (float)m.leaf_hi[l];
    const float yc = fminf(fmaxf(y, lo), hi);  // y is never NaN
    return (uint32_t)yc;  // yc >= 0: truncation is floor
}

// Cooperative copy of the model into LDS (all threads of the block; the caller
// puts a barrier after it).
template <int NT>
__device__ __forceinline__ void rmi_to_lds(tj_rmi_t* dst, const tj_rmi_t* __restrict__ src)
{
    constexpr int W = (int)(sizeof(tj_rmi_t) / 16);
    const uint4* s = (const uint4*)src;
    uint4* d = (uint4*)dst;
    for (int i = threadIdx.x; i < W; i += NT) d[i] = s[i];
}

}  // namespace tj

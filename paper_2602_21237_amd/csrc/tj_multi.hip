// tj_multi.hip - kernels of the composite-key (multi-column) sort and join.
//
// A row's key columns are the coordinates of a point in a multidimensional
// key space; packing them, most significant column first, into one unsigned
// integer is the row-major linearisation of that space, and orders rows
// lexicographically. Each column contributes the bits of (ord - column
// minimum), so a column that spans a small range costs few bits.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "tj_internal.h"

namespace tj {
namespace {

__device__ __forceinline__ uint64_t col_ord(const void* col, int kb, uint64_t i)
{
    return kb == 4 ? (uint64_t)((uint32_t)((const int32_t*)col)[i] ^ 0x80000000u)
                   : (uint64_t)((const int64_t*)col)[i] ^ 0x8000000000000000ull;
}

// packed key of row r (r < n_a: relation a, else relation b at r - n_a)
__device__ __forceinline__ uint64_t pack_row(const PackArgs& a, uint64_t r)
{
    const bool in_b = r >= a.n_a;
    const uint64_t rr = in_b ? r - a.n_a : r;
    uint64_t v = 0;
    for (int c = 0; c < a.ncols; c++) {
        const uint64_t o = col_ord(in_b ? a.col_b[c] : a.col_a[c], a.kb[c], rr) - a.min[c];
        v |= a.shift[c] < 64 ? o << a.shift[c] : 0;
    }
    return v;
}

// out[i] = packed key of row perm[i] (or of row i), as a signed key of
// out_bytes bytes whose signed order is the packed value's unsigned order
__global__ __launch_bounds__(256) void k_pack(PackArgs a, const int32_t* __restrict__ perm, uint64_t n,
                                              void* __restrict__ out, int out_bytes)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const uint64_t r = perm ? (uint64_t)(uint32_t)perm[i] : i;
        const uint64_t v = pack_row(a, r);
        if (out_bytes == 4) ((int32_t*)out)[i] = (int32_t)((uint32_t)v ^ 0x80000000u);
        else ((int64_t*)out)[i] = (int64_t)(v ^ 0x8000000000000000ull);
    }
}

// flag[i] = 1 when the row at sorted position i holds another key tuple than
// the row at i - 1 (flag[0] = 1): compared column by column
__global__ __launch_bounds__(256) void k_tuple_flags(PackArgs a, const int32_t* __restrict__ perm, uint64_t n,
                                                     uint32_t* __restrict__ flag)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        uint32_t f = 1;
        if (i > 0) {
            const uint64_t r = (uint32_t)perm[i], q = (uint32_t)perm[i - 1];
            f = 0;
            for (int c = 0; c < a.ncols; c++) {
                const void* cr = r >= a.n_a ? a.col_b[c] : a.col_a[c];
                const void* cq = q >= a.n_a ? a.col_b[c] : a.col_a[c];
                const uint64_t x = col_ord(cr, a.kb[c], r >= a.n_a ? r - a.n_a : r);
                const uint64_t y = col_ord(cq, a.kb[c], q >= a.n_a ? q - a.n_a : q);
                f |= x != y;
            }
        }
        flag[i] = f;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather(const T* __restrict__ in, const int32_t* __restrict__ perm,
                                                uint64_t n, T* __restrict__ out)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        out[i] = in[(uint32_t)perm[i]];
}

__global__ __launch_bounds__(256) void k_iota(int32_t* __restrict__ out, uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        out[i] = (int32_t)i;
}

// dst[perm[i]] = src[i]
__global__ __launch_bounds__(256) void k_scatter_back(const uint32_t* __restrict__ src,
                                                      const int32_t* __restrict__ perm, uint64_t n,
                                                      int32_t* __restrict__ dst)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        dst[(uint32_t)perm[i]] = (int32_t)src[i];
}

// Inclusive prefix sum of uint32 values in three launches: per-block totals,
// an exclusive scan of the totals in one block, then each block's own scan
// plus its offset. SCAN_ITEMS values per block.
constexpr int SCAN_NT = 256, SCAN_PER = 16, SCAN_ITEMS = SCAN_NT * SCAN_PER;

__device__ __forceinline__ uint32_t block_incl_scan_u32(uint32_t v, uint32_t* tmp, uint32_t* total)
{
    const uint32_t l = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
        if (l >= (uint32_t)d) x += y;
    }
    if (l == 63) tmp[w] = x;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_NT / 64; i++) {
        off += (uint32_t)i < w ? tmp[i] : 0u;
        tot += tmp[i];
    }
    __syncthreads();
    *total = tot;
    return x + off;
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_sums(const uint32_t* __restrict__ in, uint64_t n,
                                                       uint32_t* __restrict__ sums)
{
    __shared__ uint32_t tmp[SCAN_NT / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_ITEMS;
    uint32_t s = 0;
    for (int k = 0; k < SCAN_PER; k++) {
        const uint64_t i = b0 + (uint64_t)threadIdx.x * SCAN_PER + k;
        s += i < n ? in[i] : 0u;
    }
    uint32_t tot;
    (void)block_incl_scan_u32(s, tmp, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_offsets(uint32_t* __restrict__ sums, uint32_t nb)
{
    __shared__ uint32_t tmp[SCAN_NT / 64];
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += SCAN_NT) {  // uniform trip count
        const uint32_t b = b0 + threadIdx.x;
        const uint32_t v = b < nb ? sums[b] : 0u;
        uint32_t tot;
        const uint32_t inc = block_incl_scan_u32(v, tmp, &tot);
        if (b < nb) sums[b] = carry + inc - v;  // exclusive
        carry += tot;
    }
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_apply(const uint32_t* __restrict__ in, uint64_t n,
                                                        const uint32_t* __restrict__ sums,
                                                        uint32_t* __restrict__ out)
{
    __shared__ uint32_t tmp[SCAN_NT / 64];
    const uint64_t b0 = (uint64_t)blockIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_PER];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        const uint64_t i = b0 + (uint64_t)threadIdx.x * SCAN_PER + k;
        v[k] = i < n ? in[i] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_incl_scan_u32(s, tmp, &tot) - s + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SCAN_PER; k++) {
        const uint64_t i = b0 + (uint64_t)threadIdx.x * SCAN_PER + k;
        run += v[k];
        if (i < n) out[i] = run;
    }
}

inline uint32_t grid_for(uint64_t n)
{
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

hipError_t launch_pack(const PackArgs& a, const int32_t* perm, uint64_t n, void* out, int out_bytes, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(grid_for(n)), dim3(256), 0, st, a, perm, n, out, out_bytes);
    return hipGetLastError();
}

hipError_t launch_tuple_flags(const PackArgs& a, const int32_t* perm, uint64_t n, uint32_t* flag, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tuple_flags, dim3(grid_for(n)), dim3(256), 0, st, a, perm, n, flag);
    return hipGetLastError();
}

hipError_t launch_gather(int elem_bytes, const void* in, const int32_t* perm, uint64_t n, void* out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    if (elem_bytes == 4)
        hipLaunchKernelGGL(k_gather<int32_t>, dim3(grid_for(n)), dim3(256), 0, st, (const int32_t*)in, perm, n,
                           (int32_t*)out);
    else
        hipLaunchKernelGGL(k_gather<int64_t>, dim3(grid_for(n)), dim3(256), 0, st, (const int64_t*)in, perm, n,
                           (int64_t*)out);
    return hipGetLastError();
}

hipError_t launch_iota(int32_t* out, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_iota, dim3(grid_for(n)), dim3(256), 0, st, out, n);
    return hipGetLastError();
}

hipError_t launch_scatter_back(const uint32_t* src, const int32_t* perm, uint64_t n, int32_t* dst, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_back, dim3(grid_for(n)), dim3(256), 0, st, src, perm, n, dst);
    return hipGetLastError();
}

uint64_t scan_scratch_words(uint64_t n) { return (n + SCAN_ITEMS - 1) / SCAN_ITEMS + 1; }

hipError_t launch_incl_scan(const uint32_t* in, uint64_t n, uint32_t* scratch, uint32_t* out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint64_t nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
    if (nb > 0xffffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_sums, dim3((uint32_t)nb), dim3(SCAN_NT), 0, st, in, n, scratch);
    hipLaunchKernelGGL(k_scan_offsets, dim3(1), dim3(SCAN_NT), 0, st, scratch, (uint32_t)nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((uint32_t)nb), dim3(SCAN_NT), 0, st, in, n, (const uint32_t*)scratch, out);
    return hipGetLastError();
}

}  // namespace tj

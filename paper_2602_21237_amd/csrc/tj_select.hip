// tj_select.hip - kernels of the execution-time path selection: a
// HyperLogLog sketch of a key column (Flajolet, Fusy, Gandouet, Meunier 2007,
// with a 64-bit hash as in Heule, Nunkesser, Hall 2013).
//
// A key k (int32 keys sign-extended to int64) is hashed by the output
// function of SplitMix64 (Steele, Lea, Flood 2014) applied to the state
// (k + gamma) mod 2^64, so the hash of k is the first output of a SplitMix64
// generator seeded with k. With p = 14 index bits, register
// idx = h >> 50 takes the rank of the remaining 50 bits: the position of
// their leading one bit, counted from 1, or 51 when they are all zero.
// Registers hold the maximum rank seen, 0 for none.
//
// One pass over the column: each block keeps the 16384 registers of its own
// slice of rows in LDS (ds_max per row) and writes them to a per-block slab;
// a fold kernel takes the maximum over groups of slabs (many blocks, four
// registers per 4-byte load), a merge kernel over the groups (per relation,
// and of the two relations for their union) that also counts each wave's
// register values by ballots, and a one-block kernel sums those counts into
// the histogram the host turns into estimates. No atomics
// reach HBM, so the result does not depend on block scheduling.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "tj_internal.h"
#include "tj_select.h"

namespace tj {
namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// A 16-byte streaming load: the keys are read once, so they are not kept in
// the caches.
__device__ __forceinline__ uint4 ld_stream(const uint4* p)
{
    const u32x4 v = __builtin_nontemporal_load((const u32x4*)p);
    return make_uint4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ uint32_t hll_code(uint64_t k)
{
    uint64_t z = k + kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const uint64_t w = z << HLL_P;  // the 50 rank bits, moved to the top
    const uint32_t rank = w ? (uint32_t)__clzll((long long)w) + 1u : (uint32_t)(64 - HLL_P + 1);
    return ((uint32_t)(z >> (64 - HLL_P)) << 8) | rank;  // index << 8 | rank
}

template <typename K>
__device__ __forceinline__ uint64_t key_bits(K k)
{
    return (uint64_t)(int64_t)k;
}

__device__ __forceinline__ void hll_add(uint32_t* reg, uint64_t k)
{
    const uint32_t c = hll_code(k);
    atomicMax(&reg[c >> 8], c & 0xffu);
}

// slab[blockIdx.x][j] = max rank of the rows [b0, b1) of this block at register j.
// per_block is a multiple of HLL_ROW_ALIGN rows; with VEC the keys are 16-byte
// aligned and read 16 bytes per lane.
template <typename K, bool VEC>
__global__ __launch_bounds__(HLL_THREADS) void k_hll_block(const K* __restrict__ keys, uint64_t n,
                                                          uint64_t per_block, uint8_t* __restrict__ slab)
{
    __shared__ uint32_t reg[HLL_M];
    for (uint32_t j = threadIdx.x; j < HLL_M; j += HLL_THREADS) reg[j] = 0;
    __syncthreads();
    const uint64_t b0 = (uint64_t)blockIdx.x * per_block;
    const uint64_t b1 = b0 + per_block < n ? b0 + per_block : n;
    uint64_t i = b0 + threadIdx.x;
    if (VEC && b0 < b1) {
        constexpr uint32_t E = 16 / sizeof(K);  // keys per 16-byte vector
        constexpr int U = sizeof(K) == 8 ? 4 : 2;  // 8 keys per lane in flight
        const uint4* __restrict__ vk = (const uint4*)(keys + b0);  // b0 is a multiple of E
        const uint64_t nv = (b1 - b0) / E;
        uint64_t v = threadIdx.x;
        for (; v + (uint64_t)(U - 1) * HLL_THREADS < nv; v += (uint64_t)U * HLL_THREADS) {
            uint4 x[U];
#pragma unroll
            for (int u = 0; u < U; u++) x[u] = ld_stream(vk + v + (uint64_t)u * HLL_THREADS);
#pragma unroll
            for (int u = 0; u < U; u++) {
                if (sizeof(K) == 8) {
                    hll_add(reg, ((uint64_t)x[u].y << 32) | x[u].x);
                    hll_add(reg, ((uint64_t)x[u].w << 32) | x[u].z);
                } else {
                    hll_add(reg, key_bits((int32_t)x[u].x));
                    hll_add(reg, key_bits((int32_t)x[u].y));
                    hll_add(reg, key_bits((int32_t)x[u].z));
                    hll_add(reg, key_bits((int32_t)x[u].w));
                }
            }
        }
        for (; v < nv; v += HLL_THREADS) {
            const uint4 x = ld_stream(vk + v);
            if (sizeof(K) == 8) {
                hll_add(reg, ((uint64_t)x.y << 32) | x.x);
                hll_add(reg, ((uint64_t)x.w << 32) | x.z);
            } else {
                hll_add(reg, key_bits((int32_t)x.x));
                hll_add(reg, key_bits((int32_t)x.y));
                hll_add(reg, key_bits((int32_t)x.z));
                hll_add(reg, key_bits((int32_t)x.w));
            }
        }
        i = b0 + nv * E + threadIdx.x;  // the last < E rows of the block
    } else {
        constexpr int U = 8;
        for (; i + (uint64_t)(U - 1) * HLL_THREADS < b1; i += (uint64_t)U * HLL_THREADS) {
            K k[U];
#pragma unroll
            for (int u = 0; u < U; u++) k[u] = keys[i + (uint64_t)u * HLL_THREADS];
#pragma unroll
            for (int u = 0; u < U; u++) hll_add(reg, key_bits(k[u]));
        }
    }
    for (; i < b1; i += HLL_THREADS) {
        const uint32_t c = hll_code(key_bits(keys[i]));
        atomicMax(&reg[c >> 8], c & 0xffu);
    }
    __syncthreads();
    uint8_t* out = slab + (uint64_t)blockIdx.x * HLL_M;
    for (uint32_t j = threadIdx.x; j < HLL_M; j += HLL_THREADS) out[j] = (uint8_t)reg[j];
}

__device__ __forceinline__ uint32_t max_u8x4(uint32_t a, uint32_t b)
{
    uint32_t r = 0;
#pragma unroll
    for (int s = 0; s < 32; s += 8) r |= max((a >> s) & 0xffu, (b >> s) & 0xffu) << s;
    return r;
}

// part[z][g][j] = max over the slabs b = g, g + HLL_GROUPS, ... < nb of
// relation z (0: R, 1: S) at register j; grid (HLL_M / 1024, HLL_GROUPS, 2),
// each thread four registers (one 4-byte word) of a 1024-register column.
__global__ __launch_bounds__(256) void k_hll_fold(const uint8_t* __restrict__ slab_r, uint32_t nb_r,
                                                  const uint8_t* __restrict__ slab_s, uint32_t nb_s,
                                                  uint8_t* __restrict__ part)
{
    constexpr uint32_t W = HLL_M / 4;  // words per slab
    const uint32_t col = blockIdx.x * 256 + threadIdx.x, g = blockIdx.y, z = blockIdx.z;
    const uint32_t* __restrict__ sl = (const uint32_t*)(z ? slab_s : slab_r);
    const uint32_t nb = z ? nb_s : nb_r;
    uint32_t m = 0;
    uint32_t b = g;
    for (; b + 3 * HLL_GROUPS < nb; b += 4 * HLL_GROUPS) {
        const uint32_t x0 = sl[(uint64_t)b * W + col], x1 = sl[(uint64_t)(b + HLL_GROUPS) * W + col];
        const uint32_t x2 = sl[(uint64_t)(b + 2 * HLL_GROUPS) * W + col];
        const uint32_t x3 = sl[(uint64_t)(b + 3 * HLL_GROUPS) * W + col];
        m = max_u8x4(m, max_u8x4(max_u8x4(x0, x1), max_u8x4(x2, x3)));
    }
    for (; b < nb; b += HLL_GROUPS) m = max_u8x4(m, sl[(uint64_t)b * W + col]);
    ((uint32_t*)part)[((uint64_t)z * HLL_GROUPS + g) * W + col] = m;
}

// regs[0][j] = max over R's groups, regs[1][j] = over S's, regs[2][j] = both;
// whist[wave][a][r] = registers of array a holding rank r among the wave's 64
// (lane r counts rank r by one ballot per rank; grid HLL_M / 256 exactly).
__global__ __launch_bounds__(256) void k_hll_merge(const uint8_t* __restrict__ part, uint8_t* __restrict__ regs,
                                                   uint32_t* __restrict__ whist)
{
    const uint32_t j = blockIdx.x * 256 + threadIdx.x;
    uint32_t mr = 0, ms = 0;
#pragma unroll
    for (uint32_t g = 0; g < HLL_GROUPS; g++) {
        mr = max(mr, (uint32_t)part[(uint64_t)g * HLL_M + j]);
        ms = max(ms, (uint32_t)part[(uint64_t)(HLL_GROUPS + g) * HLL_M + j]);
    }
    regs[j] = (uint8_t)mr;
    regs[HLL_M + j] = (uint8_t)ms;
    const uint32_t mu = max(mr, ms);
    regs[2 * HLL_M + j] = (uint8_t)mu;
    const uint32_t lane = threadIdx.x & 63;
    uint32_t cr = 0, cs = 0, cu = 0;
    for (uint32_t r = 0; r <= (uint32_t)(64 - HLL_P + 1); r++) {
        const uint32_t a = (uint32_t)__popcll(__ballot(mr == r));
        const uint32_t b = (uint32_t)__popcll(__ballot(ms == r));
        const uint32_t c = (uint32_t)__popcll(__ballot(mu == r));
        if (lane == r) {
            cr = a;
            cs = b;
            cu = c;
        }
    }
    uint32_t* wh = whist + (uint64_t)(j / 64) * 3 * HLL_BINS;
    wh[lane] = cr;
    wh[HLL_BINS + lane] = cs;
    wh[2 * HLL_BINS + lane] = cu;
}

// hist[a][r] = number of registers of array a (R, S, union) holding rank r:
// the sum of the HLL_M / 64 per-wave counts; one thread per (a, r)
__global__ __launch_bounds__(3 * HLL_BINS) void k_hll_hist(const uint32_t* __restrict__ whist,
                                                           uint32_t* __restrict__ hist)
{
    uint32_t t = 0;
    for (uint32_t w = 0; w < HLL_M / 64; w++) t += whist[(uint64_t)w * 3 * HLL_BINS + threadIdx.x];
    hist[threadIdx.x] = t;
}

}  // namespace

// Rows per block: n split evenly over the blocks, rounded up to whole
// HLL_ROW_ALIGN rows, so every block starts on a 16-byte boundary of an
// aligned column; the block count then covers n exactly.
uint64_t hll_rows_per_block(uint64_t n)
{
    if (n == 0) return HLL_ROW_ALIGN;
    uint64_t b = (n + HLL_MIN_ROWS_PER_BLOCK - 1) / HLL_MIN_ROWS_PER_BLOCK;
    if (b > HLL_MAX_BLOCKS) b = HLL_MAX_BLOCKS;
    const uint64_t per = (n + b - 1) / b;
    return (per + HLL_ROW_ALIGN - 1) / HLL_ROW_ALIGN * HLL_ROW_ALIGN;
}

uint32_t hll_blocks(uint64_t n)
{
    if (n == 0) return 0;
    const uint64_t per = hll_rows_per_block(n);
    return (uint32_t)((n + per - 1) / per);
}

hipError_t launch_hll_block(int kb, const void* keys, uint64_t n, uint8_t* slab, hipStream_t st)
{
    const uint32_t nb = hll_blocks(n);
    if (nb == 0) return hipSuccess;
    const uint64_t per = hll_rows_per_block(n);
    const bool vec = ((uintptr_t)keys % 16) == 0;
    if (kb == 4) {
        if (vec)
            hipLaunchKernelGGL((k_hll_block<int32_t, true>), dim3(nb), dim3(HLL_THREADS), 0, st,
                               (const int32_t*)keys, n, per, slab);
        else
            hipLaunchKernelGGL((k_hll_block<int32_t, false>), dim3(nb), dim3(HLL_THREADS), 0, st,
                               (const int32_t*)keys, n, per, slab);
    } else {
        if (vec)
            hipLaunchKernelGGL((k_hll_block<int64_t, true>), dim3(nb), dim3(HLL_THREADS), 0, st,
                               (const int64_t*)keys, n, per, slab);
        else
            hipLaunchKernelGGL((k_hll_block<int64_t, false>), dim3(nb), dim3(HLL_THREADS), 0, st,
                               (const int64_t*)keys, n, per, slab);
    }
    return hipGetLastError();
}

hipError_t launch_hll_finish(const uint8_t* slab_r, uint32_t nb_r, const uint8_t* slab_s, uint32_t nb_s,
                             uint8_t* part, uint8_t* regs, uint32_t* whist, uint32_t* hist, hipStream_t st)
{
    hipLaunchKernelGGL(k_hll_fold, dim3(HLL_M / 1024, HLL_GROUPS, 2), dim3(256), 0, st, slab_r, nb_r, slab_s, nb_s,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hll_merge, dim3(HLL_M / 256), dim3(256), 0, st, (const uint8_t*)part, regs, whist);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hll_hist, dim3(1), dim3(3 * HLL_BINS), 0, st, (const uint32_t*)whist, hist);
    return hipGetLastError();
}

}  // namespace tj

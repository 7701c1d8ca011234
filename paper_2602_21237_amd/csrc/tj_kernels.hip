// tj_kernels.hip - gfx950 kernels of the tensor-path sort and equi-join.
//
// Everything here is integer work bound by memory traffic (the paper places
// the cost of joins and sorts in data movement and intermediate results, not
// arithmetic: Sec. I, Sec. II.C), so no matrix cores are used. The building
// blocks are wave64 primitives:
//   - ballot-based match: lanes holding the same digit find each other with one
//     ballot per digit bit, which gives each row its stable rank among equal
//     digits in the wavefront;
//   - DPP prefix sums (row_shr 1/2/4/8, row_bcast 15/31) for offsets;
//   - LDS staging so that rows leave a tile as per-digit runs (coalesced).
//
// Keys are mapped to "ordinals" that compare as unsigned integers in the same
// order as the signed keys (flip the sign bit); digits are taken from
// (ordinal - base) so that only the bits that vary inside a bucket are used.
#include "tj_internal.h"

namespace tj {

// ---------------------------------------------------------------------------
// key <-> ordinal
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ord_of(int32_t k) { return (uint64_t)((uint32_t)k ^ 0x80000000u); }
__device__ __forceinline__ uint64_t ord_of(int64_t k) { return (uint64_t)k ^ 0x8000000000000000ull; }
template <typename K> __device__ __forceinline__ K key_of(uint64_t o);
template <> __device__ __forceinline__ int32_t key_of<int32_t>(uint64_t o)
{
    return (int32_t)((uint32_t)o ^ 0x80000000u);
}
template <> __device__ __forceinline__ int64_t key_of<int64_t>(uint64_t o)
{
    return (int64_t)(o ^ 0x8000000000000000ull);
}

// ---------------------------------------------------------------------------
// wave64 primitives
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// number of set bits of m in lanes below this lane
__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t lane_id() { return mbcnt(~0ull); }

// Inclusive prefix sum across the 64 lanes with DPP: shifts of 1, 2, 4, 8
// inside each row of 16 lanes, then row_bcast:15 carries row totals into rows
// 1 and 3 and row_bcast:31 carries the first half's total into rows 2 and 3.
// Lanes whose DPP source is out of range (or whose row is masked off) read the
// `old` operand, 0, so every step is v += shifted-or-zero.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v)
{
    const uint32_t l = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t t = __shfl_up(v, (unsigned)d, 64);
        if (l >= (uint32_t)d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    return v;
}

__device__ __forceinline__ uint64_t wave_min64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t t = __shfl_xor(v, d, 64);
        v = t < v ? t : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        uint64_t t = __shfl_xor(v, d, 64);
        v = t > v ? t : v;
    }
    return v;
}

// Exclusive prefix of one value per thread over the block (NT threads);
// `tmp` holds NT/64 words of LDS. Returns the prefix; *total gets the sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* tmp, uint32_t* total)
{
    constexpr int NW = NT / 64;
    const uint32_t w = threadIdx.x / 64;
    uint32_t inc = wave_incl_scan(v);
    if ((threadIdx.x & 63) == 63) tmp[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        uint32_t t = tmp[i];
        off += ((uint32_t)i < w) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

template <int NT>
__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t* tmp)
{
    constexpr int NW = NT / 64;
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0) tmp[threadIdx.x / 64] = v;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) tot += tmp[i];
    __syncthreads();
    return tot;
}

// Stable rank of one row per lane among the rows of this wavefront with the
// same digit: rows of earlier rounds (counted in this wave's private LDS
// histogram `hist`) and lower lanes of this round. The lanes sharing a digit
// are found with one ballot per digit bit. Invalid lanes take no part.
__device__ __forceinline__ uint32_t wave_rank(uint32_t d, bool valid, int nbits, uint32_t* hist)
{
    uint64_t peers = ballot(valid);
    for (int b = 0; b < nbits; b++) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = ballot(bit);
        peers &= bit ? m : ~m;
    }
    const uint32_t below = mbcnt(peers);
    uint32_t base = 0;
    if (valid) base = hist[d];
    if (valid && below == 0) hist[d] = base + (uint32_t)__popcll(peers);
    return base + below;
}

// Turns per-wave digit counts whist[w * nbins_stride + d] into per-wave
// exclusive offsets inside the tile: texcl[d] = rows of smaller digits,
// whist[w][d] = rows of digit d in waves before w; tcount[d] = rows of digit d.
// Returns the tile's row total. Ends with a barrier.
template <int NT, int NBINS>
__device__ __forceinline__ uint32_t tile_scan(uint32_t* whist, uint32_t* tcount, uint32_t* texcl,
                                              uint32_t* tmp)
{
    constexpr int NW = NT / 64;
    constexpr int DPT = (NBINS + NT - 1) / NT;
    uint32_t sums[DPT];
    uint32_t local = 0;
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const int d = threadIdx.x * DPT + i;
        uint32_t s = 0;
        if (d < NBINS) {
#pragma unroll
            for (int w = 0; w < NW; w++) {
                const uint32_t v = whist[w * NBINS + d];
                whist[w * NBINS + d] = s;
                s += v;
            }
            tcount[d] = s;
        }
        sums[i] = s;
        local += s;
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<NT>(local, tmp, &tot);
#pragma unroll
    for (int i = 0; i < DPT; i++) {
        const int d = threadIdx.x * DPT + i;
        if (d < NBINS) texcl[d] = ex;
        ex += sums[i];
    }
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t* p, uint64_t n, uint64_t v)
{
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t n, uint64_t v, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

__global__ void k_wave_scan_test(const uint32_t* in, uint32_t* out, uint64_t n)
{
    const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint32_t v = i < n ? in[i] : 0u;
    const uint32_t s = wave_incl_scan(v);
    if (i < n) out[i] = s;
}

hipError_t launch_wave_scan_test(const uint32_t* in, uint32_t* out, uint64_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_wave_scan_test, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// range probe: minimum and maximum ordinal over one or two key columns
// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(256) void k_probe(const K* __restrict__ a, uint64_t na,
                                               const K* __restrict__ b, uint64_t nb,
                                               uint64_t* __restrict__ minmax)
{
    __shared__ uint64_t smin[4], smax[4];
    uint64_t mn = ~0ull, mx = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < na; i += stride) {
        const uint64_t o = ord_of(a[i]);
        mn = o < mn ? o : mn;
        mx = o > mx ? o : mx;
    }
    for (uint64_t i = t0; i < nb; i += stride) {
        const uint64_t o = ord_of(b[i]);
        mn = o < mn ? o : mn;
        mx = o > mx ? o : mx;
    }
    mn = wave_min64(mn);
    mx = wave_max64(mx);
    if ((threadIdx.x & 63) == 0) {
        smin[threadIdx.x / 64] = mn;
        smax[threadIdx.x / 64] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < 4; i++) {
            mn = smin[i] < mn ? smin[i] : mn;
            mx = smax[i] > mx ? smax[i] : mx;
        }
        atomicMin((unsigned long long*)&minmax[0], (unsigned long long)mn);
        atomicMax((unsigned long long*)&minmax[1], (unsigned long long)mx);
    }
}

hipError_t launch_probe(int key_bytes, const void* a, uint64_t na, const void* b, uint64_t nb,
                        uint64_t* minmax, hipStream_t st)
{
    hipError_t e = launch_fill_u64(minmax, 1, ~0ull, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u64(minmax + 1, 1, 0ull, st);
    if (e != hipSuccess) return e;
    const uint64_t n = na > nb ? na : nb;
    uint64_t blocks = (n + 256 * 16 - 1) / (256 * 16);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_probe<int32_t>, dim3((uint32_t)blocks), dim3(256), 0, st,
                           (const int32_t*)a, na, (const int32_t*)b, nb, minmax);
    else
        hipLaunchKernelGGL(k_probe<int64_t>, dim3((uint32_t)blocks), dim3(256), 0, st,
                           (const int64_t*)a, na, (const int64_t*)b, nb, minmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// radix histogram: per chunk, the digit counts of its rows (and, per group
// and digit, the smallest and largest ordinal, so that every child bucket
// knows its exact key range and single-key buckets are recognised)
// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(PART_THREADS) void k_hist(const ChunkDesc* __restrict__ chunks,
                                                       const GroupDesc* __restrict__ groups,
                                                       BufSet bufs, uint32_t* __restrict__ hist,
                                                       uint64_t* __restrict__ gmin,
                                                       uint64_t* __restrict__ gmax)
{
    __shared__ uint32_t cnt[NB];
    __shared__ uint64_t mn[NB], mx[NB];
    const ChunkDesc ch = chunks[blockIdx.x];
    const GroupDesc g = groups[ch.group];
    const K* __restrict__ src = (const K*)bufs.key[g.src][g.side] + ch.start;
    const uint32_t nbins = 1u << g.bits;
    for (uint32_t d = threadIdx.x; d < nbins; d += PART_THREADS) {
        cnt[d] = 0;
        mn[d] = ~0ull;
        mx[d] = 0;
    }
    __syncthreads();
    constexpr int U = 4;
    for (uint32_t q0 = threadIdx.x; q0 < ch.len; q0 += PART_THREADS * U) {
        K k[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t q = q0 + u * PART_THREADS;
            k[u] = q < ch.len ? src[q] : K(0);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t q = q0 + u * PART_THREADS;
            const uint64_t o = ord_of(k[u]);
            if (q < ch.len && o >= g.flo && o <= g.fhi) {
                const uint32_t d = (uint32_t)((o - g.base) >> g.shift) & (nbins - 1u);
                atomicAdd(&cnt[d], 1u);
                atomicMin((unsigned long long*)&mn[d], (unsigned long long)o);
                atomicMax((unsigned long long*)&mx[d], (unsigned long long)o);
            }
        }
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < nbins; d += PART_THREADS) {
        hist[(uint64_t)blockIdx.x * NB + d] = cnt[d];
        if (cnt[d]) {
            atomicMin((unsigned long long*)&gmin[g.child0 + d], (unsigned long long)mn[d]);
            atomicMax((unsigned long long*)&gmax[g.child0 + d], (unsigned long long)mx[d]);
        }
    }
}

hipError_t launch_hist(int key_bytes, const ChunkDesc* chunks, uint32_t nchunks,
                       const GroupDesc* groups, BufSet bufs, uint32_t* hist, uint64_t* gmin,
                       uint64_t* gmax, hipStream_t st)
{
    if (nchunks == 0) return hipSuccess;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_hist<int32_t>, dim3(nchunks), dim3(PART_THREADS), 0, st, chunks, groups,
                           bufs, hist, gmin, gmax);
    else
        hipLaunchKernelGGL(k_hist<int64_t>, dim3(nchunks), dim3(PART_THREADS), 0, st, chunks, groups,
                           bufs, hist, gmin, gmax);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// offset scan, two levels. Level 1 (one block per scan block of <= CBLOCK
// chunks): hist[c][d] becomes the exclusive prefix of digit d over the scan
// block's earlier chunks; cbsum[b][d] the scan block's total. Level 2 (one
// block per group): cbsum[b][d] becomes the prefix over the group's earlier
// scan blocks, ccount[d] the group's digit totals and cstart[d] the first
// destination row of digit d (digit-major, so buckets are in key order).
// A row of chunk c with digit d and rank r inside the chunk goes to
// cstart[d] + cbsum[b][d] + hist[c][d] + r.
// ---------------------------------------------------------------------------
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_DPT = NB / SCAN_THREADS;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_l1(const CBlockDesc* __restrict__ cblocks,
                                                          uint32_t* __restrict__ hist,
                                                          uint32_t* __restrict__ cbsum)
{
    const CBlockDesc cb = cblocks[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_DPT; i++) {
        const uint32_t d = threadIdx.x + i * SCAN_THREADS;
        uint32_t run = 0;
        uint32_t v[CBLOCK];
#pragma unroll
        for (int c = 0; c < CBLOCK; c++)
            v[c] = (uint32_t)c < cb.nchunks ? hist[(uint64_t)(cb.chunk0 + c) * NB + d] : 0u;
#pragma unroll
        for (int c = 0; c < CBLOCK; c++) {
            if ((uint32_t)c < cb.nchunks) hist[(uint64_t)(cb.chunk0 + c) * NB + d] = run;
            run += v[c];
        }
        cbsum[(uint64_t)blockIdx.x * NB + d] = run;
    }
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_l2(const GroupDesc* __restrict__ groups,
                                                          uint32_t* __restrict__ cbsum,
                                                          uint32_t* __restrict__ ccount,
                                                          uint64_t* __restrict__ cstart)
{
    __shared__ uint32_t tmp[SCAN_THREADS / 64];
    const GroupDesc g = groups[blockIdx.x];
    const uint32_t nbins = 1u << g.bits;
    uint32_t tot[SCAN_DPT];
    uint32_t local = 0;
#pragma unroll
    for (int i = 0; i < SCAN_DPT; i++) {
        // contiguous digits per thread keep the block scan in digit order
        const uint32_t d = threadIdx.x * SCAN_DPT + i;
        uint32_t run = 0;
        for (uint32_t b = 0; b < g.ncblocks; b++) {
            const uint64_t at = (uint64_t)(g.cblock0 + b) * NB + d;
            const uint32_t v = cbsum[at];
            cbsum[at] = run;
            run += v;
        }
        tot[i] = d < nbins ? run : 0u;
        local += tot[i];
    }
    uint32_t all;
    uint64_t ex = block_excl_scan<SCAN_THREADS>(local, tmp, &all);
#pragma unroll
    for (int i = 0; i < SCAN_DPT; i++) {
        const uint32_t d = threadIdx.x * SCAN_DPT + i;
        if (d < nbins) {
            ccount[g.child0 + d] = tot[i];
            cstart[g.child0 + d] = g.dst_start + ex;
        }
        ex += tot[i];
    }
}

hipError_t launch_scan(const CBlockDesc* cblocks, uint32_t ncblocks, const GroupDesc* groups,
                       uint32_t ngroups, uint32_t* hist, uint32_t* cbsum, uint32_t* ccount,
                       uint64_t* cstart, hipStream_t st)
{
    if (ncblocks == 0 || ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_l1, dim3(ncblocks), dim3(SCAN_THREADS), 0, st, cblocks, hist, cbsum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_l2, dim3(ngroups), dim3(SCAN_THREADS), 0, st, groups, cbsum, ccount, cstart);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stable LDS-staged scatter. Each block walks its chunk in tiles of
// PART_TILE rows. Per tile: rows are loaded coalesced, ranked within their
// wave by ballot match, offset across waves and digits (tile_scan), staged in
// LDS grouped by digit, and then written out as per-digit runs.
// Wave w of the tile owns rows [w*ITEMS*64, (w+1)*ITEMS*64); round r of a wave
// covers 64 consecutive rows, so (wave, round, lane) is input order and the
// partition is stable.
// ---------------------------------------------------------------------------
template <typename K, bool RIDS, bool WKEYS>
__global__ __launch_bounds__(PART_THREADS) void k_scatter(const ChunkDesc* __restrict__ chunks,
                                                          const GroupDesc* __restrict__ groups,
                                                          const uint32_t* __restrict__ hist,
                                                          const uint32_t* __restrict__ cbsum,
                                                          const uint64_t* __restrict__ cstart,
                                                          BufSet bufs)
{
    constexpr int NT = PART_THREADS, KI = PART_ITEMS, NW = NT / 64, TILE = PART_TILE;
    __shared__ uint32_t whist[NW * NB];
    __shared__ uint32_t tcount[NB], texcl[NB], run[NB];
    __shared__ uint32_t tmp[NW];
    __shared__ K skey[TILE];
    __shared__ int32_t srid[RIDS ? TILE : 1];
    __shared__ uint16_t sdig[TILE];

    const ChunkDesc ch = chunks[blockIdx.x];
    const GroupDesc g = groups[ch.group];
    const K* __restrict__ src_k = (const K*)bufs.key[g.src][g.side] + ch.start;
    const int32_t* __restrict__ src_r = bufs.rid[g.src][g.side] + ch.start;
    K* __restrict__ dst_k = (K*)bufs.key[g.dst][g.side];
    int32_t* __restrict__ dst_r = (int32_t*)bufs.rid[g.dst][g.side];
    const uint32_t nbins = 1u << g.bits;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;

    for (uint32_t d = threadIdx.x; d < NB; d += NT)
        run[d] = d < nbins ? (uint32_t)(cstart[g.child0 + d] + cbsum[(uint64_t)ch.cblock * NB + d] +
                                        hist[(uint64_t)blockIdx.x * NB + d])
                           : 0u;
    for (uint32_t t0 = 0; t0 < ch.len; t0 += TILE) {
        K key[KI];
        int32_t rid[KI];
        uint32_t dig[KI], rk[KI];
        bool val[KI];
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = t0 + (w * KI + r) * 64 + l;
            val[r] = q < ch.len;
            key[r] = val[r] ? src_k[q] : K(0);
            if (RIDS) rid[r] = val[r] ? src_r[q] : 0;
        }
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint64_t o = ord_of(key[r]);
            val[r] = val[r] && o >= g.flo && o <= g.fhi;
            dig[r] = val[r] ? (uint32_t)((o - g.base) >> g.shift) & (nbins - 1u) : 0u;
        }
        for (uint32_t i = l; i < NB; i += 64) whist[w * NB + i] = 0;
#pragma unroll
        for (int r = 0; r < KI; r++) rk[r] = wave_rank(dig[r], val[r], (int)g.bits, &whist[w * NB]);
        __syncthreads();
        const uint32_t nvalid = tile_scan<NT, NB>(whist, tcount, texcl, tmp);
#pragma unroll
        for (int r = 0; r < KI; r++) {
            if (val[r]) {
                const uint32_t d = dig[r];
                const uint32_t p = texcl[d] + whist[w * NB + d] + rk[r];
                skey[p] = key[r];
                if (RIDS) srid[p] = rid[r];
                sdig[p] = (uint16_t)d;
            }
        }
        __syncthreads();
        for (uint32_t p = threadIdx.x; p < nvalid; p += NT) {
            const uint32_t d = sdig[p];
            const uint32_t dst = run[d] + (p - texcl[d]);
            if (WKEYS) dst_k[dst] = skey[p];
            if (RIDS) dst_r[dst] = srid[p];
        }
        __syncthreads();
        for (uint32_t d = threadIdx.x; d < NB; d += NT) run[d] += tcount[d];
        __syncthreads();
    }
}

hipError_t launch_scatter(int key_bytes, bool rids, bool keys, const ChunkDesc* chunks, uint32_t nchunks,
                          const GroupDesc* groups, const uint32_t* hist, const uint32_t* cbsum,
                          const uint64_t* cstart, BufSet bufs, hipStream_t st)
{
    if (nchunks == 0) return hipSuccess;
    const dim3 grid(nchunks), block(PART_THREADS);
#define TJ_SC(K, R, W)                                                                               \
    hipLaunchKernelGGL((k_scatter<K, R, W>), grid, block, 0, st, chunks, groups, hist, cbsum, cstart, bufs)
    if (key_bytes == 4) {
        if (!keys) TJ_SC(int32_t, true, false);
        else if (rids) TJ_SC(int32_t, true, true);
        else TJ_SC(int32_t, false, true);
    } else {
        if (!keys) TJ_SC(int64_t, true, false);
        else if (rids) TJ_SC(int64_t, true, true);
        else TJ_SC(int64_t, false, true);
    }
#undef TJ_SC
    return hipGetLastError();
}

// Expansion of a single-key join range straight in the output columns.
// mode 0: dst[t] = src[t / b] for t in [0, n); mode 1: dst[t] = dst[t mod b] for t in [b, n).
__global__ __launch_bounds__(256) void k_expand(int32_t* __restrict__ dst, const int32_t* __restrict__ src,
                                                uint64_t n, uint64_t b, int mode)
{
    for (uint64_t t = blockIdx.x * 256ull + threadIdx.x; t < n; t += (uint64_t)gridDim.x * 256) {
        uint64_t i = (uint64_t)((double)t / (double)b);
        while (i * b > t) i--;
        while ((i + 1) * b <= t) i++;
        if (mode == 0) dst[t] = src[i];
        else if (t >= b) dst[t] = dst[t - i * b];
    }
}

hipError_t launch_expand(int32_t* dst, const int32_t* src, uint64_t n, uint64_t b, int mode, hipStream_t st)
{
    if (n == 0 || b == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_expand, dim3((uint32_t)blocks), dim3(256), 0, st, dst, src, n, b, mode);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-bucket LDS sort: a stable LSD radix sort, 8-bit digits, of NT*KI items
// held in registers, items exchanged through LDS after every digit. KW is the
// relative-key word: 32 bits when the bucket's keys span < 2^32, else 64.
// On return the sorted items are in lds_key / lds_idx. Padding items carry
// the all-ones key and the largest positions, so they sort last.
// ---------------------------------------------------------------------------
template <typename KW, int NT, int KI>
__device__ __forceinline__ void block_lsd_sort(KW (&key)[KI], uint16_t (&idx)[KI], int bits,
                                               KW* lds_key, uint16_t* lds_idx, uint32_t* whist,
                                               uint32_t* tcount, uint32_t* texcl, uint32_t* tmp)
{
    constexpr int NBL = 256;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    const int passes = (bits + 7) / 8;
    if (passes == 0) {
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = (w * KI + r) * 64 + l;
            lds_key[q] = key[r];
            lds_idx[q] = idx[r];
        }
        __syncthreads();
        return;
    }
    for (int p = 0; p < passes; p++) {
        const int sh = 8 * p;
        const int nb = bits - sh < 8 ? bits - sh : 8;
        const uint32_t mask = (1u << nb) - 1u;
        uint32_t dig[KI], rk[KI];
#pragma unroll
        for (int r = 0; r < KI; r++) dig[r] = (uint32_t)(key[r] >> sh) & mask;
        for (uint32_t i = l; i < NBL; i += 64) whist[w * NBL + i] = 0;
#pragma unroll
        for (int r = 0; r < KI; r++) rk[r] = wave_rank(dig[r], true, nb, &whist[w * NBL]);
        __syncthreads();
        tile_scan<NT, NBL>(whist, tcount, texcl, tmp);
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t d = dig[r];
            const uint32_t pos = texcl[d] + whist[w * NBL + d] + rk[r];
            lds_key[pos] = key[r];
            lds_idx[pos] = idx[r];
        }
        __syncthreads();
        if (p + 1 < passes) {
#pragma unroll
            for (int r = 0; r < KI; r++) {
                const uint32_t q = (w * KI + r) * 64 + l;
                key[r] = lds_key[q];
                idx[r] = lds_idx[q];
            }
        }
    }
}

constexpr int LEAF_NW = LEAF_THREADS / 64;
constexpr size_t LEAF_SCRATCH = (size_t)LEAF_NW * 256 * 4 + 2 * 256 * 4 + 64 * 8;

template <typename K, typename KW>
__global__ __launch_bounds__(LEAF_THREADS) void k_leaf_sort(const LeafDesc* __restrict__ leaves,
                                                            BufSet bufs, K* __restrict__ out_k,
                                                            int32_t* __restrict__ out_r)
{
    constexpr int NT = LEAF_THREADS, KI = LEAF_ITEMS, C = LEAF_CAP;
    __shared__ KW lds_key[C];
    __shared__ uint16_t lds_idx[C];
    __shared__ int32_t lds_rid[C];
    __shared__ uint32_t whist[LEAF_NW * 256];
    __shared__ uint32_t tcount[256], texcl[256], tmp[LEAF_NW];

    const LeafDesc L = leaves[blockIdx.x];
    const K* __restrict__ src_k = (const K*)bufs.key[L.buf][0] + L.r0;
    const int32_t* __restrict__ src_r = bufs.rid[L.buf][0] + L.r0;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    KW key[KI];
    uint16_t idx[KI];
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        if (q < L.rn) {
            key[r] = (KW)(ord_of(src_k[q]) - L.base);
            lds_rid[q] = src_r[q];
        } else {
            key[r] = (KW)~(KW)0;
        }
        idx[r] = (uint16_t)q;
    }
    block_lsd_sort<KW, NT, KI>(key, idx, (int)L.bits, lds_key, lds_idx, whist, tcount, texcl, tmp);
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        if (q < L.rn) {
            out_k[L.out + q] = key_of<K>(L.base + (uint64_t)lds_key[q]);
            out_r[L.out + q] = lds_rid[lds_idx[q]];
        }
    }
}

hipError_t launch_leaf_sort(int key_bytes, bool wide, const LeafDesc* leaves, uint32_t n,
                            BufSet bufs, void* out_k, int32_t* out_r, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 grid(n), block(LEAF_THREADS);
    if (key_bytes == 4) {
        if (wide)
            hipLaunchKernelGGL((k_leaf_sort<int32_t, uint64_t>), grid, block, 0, st, leaves, bufs, (int32_t*)out_k, out_r);
        else
            hipLaunchKernelGGL((k_leaf_sort<int32_t, uint32_t>), grid, block, 0, st, leaves, bufs, (int32_t*)out_k, out_r);
    } else {
        if (wide)
            hipLaunchKernelGGL((k_leaf_sort<int64_t, uint64_t>), grid, block, 0, st, leaves, bufs, (int64_t*)out_k, out_r);
        else
            hipLaunchKernelGGL((k_leaf_sort<int64_t, uint32_t>), grid, block, 0, st, leaves, bufs, (int64_t*)out_k, out_r);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// per-bucket join. The block loads R's rows (positions 0..rn-1) and then S's
// rows (rn..rn+sn-1) of its co-partition and sorts them together, stably, by
// key: every key then forms one run [R rows in input order][S rows in input
// order]. A run with a R rows and b S rows contributes a*b pairs; R row i of
// the run owns the b consecutive output slots of its pairs, so the output is
// key-ascending, R-major, S in input order.
// ---------------------------------------------------------------------------
template <typename KW>
__device__ __forceinline__ uint32_t lds_lower_bound(const KW* a, uint32_t lo, uint32_t hi, KW k)
{
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (a[m] < k) lo = m + 1; else hi = m;
    }
    return lo;
}

template <typename KW>
__device__ __forceinline__ uint32_t lds_upper_bound(const KW* a, uint32_t lo, uint32_t hi, KW k)
{
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (a[m] <= k) lo = m + 1; else hi = m;
    }
    return lo;
}

template <typename K, typename KW, bool MAT>
__global__ __launch_bounds__(LEAF_THREADS) void k_leaf_join(const LeafDesc* __restrict__ leaves,
                                                            BufSet bufs, uint64_t* __restrict__ counts,
                                                            int32_t* __restrict__ out_r,
                                                            int32_t* __restrict__ out_s)
{
    constexpr int NT = LEAF_THREADS, KI = LEAF_ITEMS, C = LEAF_CAP;
    // key array; after the run analysis its storage holds s0 (and, when KW is
    // 64-bit, the pair offsets E as well)
    __shared__ KW lds_key[C];
    __shared__ uint16_t lds_idx[C];
    __shared__ int32_t lds_rid[MAT ? C : 1];
    __shared__ uint32_t lds_e_own[(MAT && sizeof(KW) == 4) ? C : 1];
    __shared__ uint32_t whist[LEAF_NW * 256];
    __shared__ uint32_t tcount[256], texcl[256], tmp[LEAF_NW];
    __shared__ uint64_t tmp64[LEAF_NW];

    const LeafDesc L = leaves[blockIdx.x];
    const uint32_t n = L.rn + L.sn;
    const K* __restrict__ rk = (const K*)bufs.key[L.buf][0] + L.r0;
    const K* __restrict__ sk = (const K*)bufs.key[L.buf][1] + L.s0;
    const int32_t* __restrict__ rr = bufs.rid[L.buf][0] + L.r0;
    const int32_t* __restrict__ sr = bufs.rid[L.buf][1] + L.s0;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;

    KW key[KI];
    uint16_t idx[KI];
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        if (q < L.rn) {
            key[r] = (KW)(ord_of(rk[q]) - L.base);
            if (MAT) lds_rid[q] = rr[q];
        } else if (q < n) {
            key[r] = (KW)(ord_of(sk[q - L.rn]) - L.base);
            if (MAT) lds_rid[q] = sr[q - L.rn];
        } else {
            key[r] = (KW)~(KW)0;
        }
        idx[r] = (uint16_t)q;
    }
    block_lsd_sort<KW, NT, KI>(key, idx, (int)L.bits, lds_key, lds_idx, whist, tcount, texcl, tmp);

    if (!MAT) {
        uint64_t c = 0;
        for (uint32_t p = threadIdx.x; p < n; p += NT) {
            if (lds_idx[p] >= L.rn) continue;
            const KW k = lds_key[p];
            const bool last_r = p + 1 == n || lds_idx[p + 1] >= L.rn || lds_key[p + 1] != k;
            if (!last_r) continue;
            const uint32_t lo = lds_lower_bound<KW>(lds_key, 0, p, k);
            const uint32_t e = lds_upper_bound<KW>(lds_key, p + 1, n, k);
            c += (uint64_t)(p + 1 - lo) * (uint64_t)(e - (p + 1));
        }
        c = block_sum64<NT>(c, tmp64);
        if (threadIdx.x == 0) counts[blockIdx.x] = c;
        return;
    }

    // Materialise. Phase A: for each R item, the S part of its run [s0, e).
    uint32_t bcnt[KI], s0v[KI];
    uint32_t local = 0;
#pragma unroll
    for (int i = 0; i < KI; i++) {
        const uint32_t p = threadIdx.x * KI + i;
        bcnt[i] = 0;
        s0v[i] = 0;
        if (p < n && lds_idx[p] < L.rn) {
            const KW k = lds_key[p];
            const uint32_t e = lds_upper_bound<KW>(lds_key, p + 1, n, k);
            // first S item of the run: S items follow the run's R items
            uint32_t lo = p + 1, hi = e;
            while (lo < hi) {
                const uint32_t m = (lo + hi) >> 1;
                if (lds_idx[m] < L.rn) lo = m + 1; else hi = m;
            }
            s0v[i] = lo;
            bcnt[i] = e - lo;
        }
        local += bcnt[i];
    }
    uint32_t total;
    uint32_t ex = block_excl_scan<NT>(local, tmp, &total);  // contains barriers: keys no longer read
    uint32_t* lds_s0 = (uint32_t*)lds_key;
    uint32_t* lds_e = sizeof(KW) == 4 ? lds_e_own : (uint32_t*)lds_key + C;
#pragma unroll
    for (int i = 0; i < KI; i++) {
        const uint32_t p = threadIdx.x * KI + i;
        lds_s0[p] = s0v[i];
        lds_e[p] = ex;
        ex += bcnt[i];
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < total; t += NT) {
        // the R item owning pair t: the last position p < n with E[p] <= t
        uint32_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const uint32_t m = (lo + hi) >> 1;
            if (lds_e[m] <= t) lo = m; else hi = m;
        }
        const uint32_t j = t - lds_e[lo];
        out_r[L.out + t] = lds_rid[lds_idx[lo]];
        out_s[L.out + t] = lds_rid[lds_idx[lds_s0[lo] + j]];
    }
}

hipError_t launch_leaf_join(int key_bytes, bool wide, bool materialize, const LeafDesc* leaves,
                            uint32_t n, BufSet bufs, uint64_t* counts, int32_t* out_r,
                            int32_t* out_s, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 grid(n), block(LEAF_THREADS);
#define TJ_LJ(K, KW, M)                                                                              \
    hipLaunchKernelGGL((k_leaf_join<K, KW, M>), grid, block, 0, st, leaves, bufs, counts, out_r, out_s)
    if (key_bytes == 4) {
        if (wide) { if (materialize) TJ_LJ(int32_t, uint64_t, true); else TJ_LJ(int32_t, uint64_t, false); }
        else      { if (materialize) TJ_LJ(int32_t, uint32_t, true); else TJ_LJ(int32_t, uint32_t, false); }
    } else {
        if (wide) { if (materialize) TJ_LJ(int64_t, uint64_t, true); else TJ_LJ(int64_t, uint64_t, false); }
        else      { if (materialize) TJ_LJ(int64_t, uint32_t, true); else TJ_LJ(int64_t, uint32_t, false); }
    }
#undef TJ_LJ
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// single-key buckets of the join: pair t of a unit with a R rows and b S rows
// is (R row t / b, S row t mod b); consecutive t are written by consecutive
// threads (coalesced). Units are flattened into one sequence of pairs and
// each block takes a fixed stretch of it.
// ---------------------------------------------------------------------------
constexpr int CROSS_THREADS = 256;
constexpr uint64_t CROSS_PER_BLOCK = 256 * 64;

__device__ __forceinline__ uint32_t find_unit(const uint64_t* pfx_base, size_t stride_words,
                                              uint32_t n, uint64_t t)
{
    // last unit u with pfx(u) <= t
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (pfx_base[(size_t)m * stride_words] <= t) lo = m; else hi = m;
    }
    return lo;
}

__global__ __launch_bounds__(CROSS_THREADS) void k_cross(const CrossDesc* __restrict__ units,
                                                         uint32_t n, uint64_t total, BufSet bufs,
                                                         int32_t* __restrict__ out_r,
                                                         int32_t* __restrict__ out_s)
{
    const uint64_t t0 = blockIdx.x * CROSS_PER_BLOCK;
    uint64_t t1 = t0 + CROSS_PER_BLOCK;
    if (t1 > total) t1 = total;
    const size_t stride = sizeof(CrossDesc) / 8;
    const uint64_t* pfx = &units[0].pfx;
    uint64_t t = t0 + threadIdx.x;
    if (t >= t1) return;
    uint32_t u = find_unit(pfx, stride, n, t);
    CrossDesc U = units[u];
    for (; t < t1; t += CROSS_THREADS) {
        while (t >= U.pfx + U.a * U.b) U = units[++u];
        const uint64_t loc = t - U.pfx;
        uint64_t i = (uint64_t)((double)loc / (double)U.b);
        while (i * U.b > loc) i--;
        while ((i + 1) * U.b <= loc) i++;
        const uint64_t j = loc - i * U.b;
        out_r[U.out + loc] = bufs.rid[U.buf][0][U.r0 + i];
        out_s[U.out + loc] = bufs.rid[U.buf][1][U.s0 + j];
    }
}

hipError_t launch_cross(const CrossDesc* units, uint32_t n, uint64_t total, BufSet bufs,
                        int32_t* out_r, int32_t* out_s, hipStream_t st)
{
    if (n == 0 || total == 0) return hipSuccess;
    const uint64_t blocks = (total + CROSS_PER_BLOCK - 1) / CROSS_PER_BLOCK;
    hipLaunchKernelGGL(k_cross, dim3((uint32_t)blocks), dim3(CROSS_THREADS), 0, st, units, n, total,
                       bufs, out_r, out_s);
    return hipGetLastError();
}

// single-key buckets of the sort that are not yet in the output columns
template <typename K>
__global__ __launch_bounds__(CROSS_THREADS) void k_copy(const CopyDesc* __restrict__ units,
                                                        uint32_t n, uint64_t total, BufSet bufs,
                                                        K* __restrict__ out_k,
                                                        int32_t* __restrict__ out_r)
{
    const uint64_t t0 = blockIdx.x * CROSS_PER_BLOCK;
    uint64_t t1 = t0 + CROSS_PER_BLOCK;
    if (t1 > total) t1 = total;
    const size_t stride = sizeof(CopyDesc) / 8;
    const uint64_t* pfx = &units[0].pfx;
    uint64_t t = t0 + threadIdx.x;
    if (t >= t1) return;
    uint32_t u = find_unit(pfx, stride, n, t);
    CopyDesc U = units[u];
    for (; t < t1; t += CROSS_THREADS) {
        while (t >= U.pfx + U.len) U = units[++u];
        const uint64_t loc = t - U.pfx;
        out_k[U.out + loc] = ((const K*)bufs.key[U.buf][0])[U.start + loc];
        out_r[U.out + loc] = bufs.rid[U.buf][0][U.start + loc];
    }
}

hipError_t launch_copy(int key_bytes, const CopyDesc* units, uint32_t n, uint64_t total,
                       BufSet bufs, void* out_k, int32_t* out_r, hipStream_t st)
{
    if (n == 0 || total == 0) return hipSuccess;
    const uint64_t blocks = (total + CROSS_PER_BLOCK - 1) / CROSS_PER_BLOCK;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_copy<int32_t>, dim3((uint32_t)blocks), dim3(CROSS_THREADS), 0, st, units, n,
                           total, bufs, (int32_t*)out_k, out_r);
    else
        hipLaunchKernelGGL(k_copy<int64_t>, dim3((uint32_t)blocks), dim3(CROSS_THREADS), 0, st, units, n,
                           total, bufs, (int64_t*)out_k, out_r);
    return hipGetLastError();
}

}  // namespace tj

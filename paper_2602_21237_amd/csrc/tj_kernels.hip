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
#include "tj_rmi.h"

#include <type_traits>

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

// Workgroup barrier that orders LDS traffic only. Blocks here never hand data
// to each other through global memory inside a launch (global reads that feed
// LDS complete before their LDS write, by data dependence), so outstanding
// global stores need not drain at a barrier; a plain __syncthreads() would wait
// for them (vmcnt(0)) and serialise store latency into every tile.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
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

// p[min(q, n - 1)], n >= 1. The load is unconditional (the clamped index
// always names a real element), so an unrolled batch of them is issued before
// the first wait; a guarded load would wait on each one in turn.
template <typename T>
__device__ __forceinline__ T ld_clamp(const T* __restrict__ p, uint64_t q, uint64_t n)
{
    return p[q < n ? q : n - 1];
}

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
    lds_barrier();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) {
        uint32_t t = tmp[i];
        off += ((uint32_t)i < w) ? t : 0u;
        tot += t;
    }
    lds_barrier();
    *total = tot;
    return off + inc - v;
}

template <int NT>
__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t* tmp)
{
    constexpr int NW = NT / 64;
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0) tmp[threadIdx.x / 64] = v;
    lds_barrier();
    uint64_t tot = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) tot += tmp[i];
    lds_barrier();
    return tot;
}

// Inclusive running maximum across the wave (same DPP pattern as the sum; 0 is
// the identity, values are non-negative).
__device__ __forceinline__ uint32_t wave_incl_max(uint32_t v)
{
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));
    return v;
}

// Maximum over the values of all threads before this one (0 for thread 0).
template <int NT>
__device__ __forceinline__ uint32_t block_excl_max(uint32_t v, uint32_t* tmp)
{
    constexpr int NW = NT / 64;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    const uint32_t inc = wave_incl_max(v);
    if (l == 63) tmp[w] = inc;
    uint32_t prev = (uint32_t)__shfl_up((int)inc, 1u, 64);
    if (l == 0) prev = 0;
    lds_barrier();
    uint32_t off = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) off = ((uint32_t)i < w && tmp[i] > off) ? tmp[i] : off;
    lds_barrier();
    return max(off, prev);
}

// Maximum over the block.
template <int NT>
__device__ __forceinline__ uint32_t block_max(uint32_t v, uint32_t* tmp)
{
    constexpr int NW = NT / 64;
    const uint32_t inc = wave_incl_max(v);
    if ((threadIdx.x & 63) == 63) tmp[threadIdx.x / 64] = inc;
    lds_barrier();
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < NW; i++) m = tmp[i] > m ? tmp[i] : m;
    lds_barrier();
    return m;
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

// Per-wave digit counters live in LDS as cnt[w * (BINS + 1) + d]; the padding
// word spreads both a wave's random digits and the column walk below across
// banks. scan_counts turns them, by one block-wide exclusive scan in
// (digit, wave) order, into offsets inside the tile:
//   cnt[w][d] = rows with a smaller digit + rows of digit d in earlier waves.
// Returns the tile's row total. Ends with a barrier.
template <int NT, int NW, int BINS>
__device__ __forceinline__ uint32_t scan_counts(uint32_t* cnt, uint32_t* tmp)
{
    constexpr int STRIDE = BINS + 1;
    constexpr int E = BINS * NW;
    constexpr int EPT = E / NT;
    static_assert(E % NT == 0, "counter matrix must split evenly over the block");
    uint32_t v[EPT];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < EPT; i++) {
        const int e = threadIdx.x * EPT + i;
        v[i] = cnt[(e % NW) * STRIDE + e / NW];
        s += v[i];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<NT>(s, tmp, &tot);
#pragma unroll
    for (int i = 0; i < EPT; i++) {
        const int e = threadIdx.x * EPT + i;
        cnt[(e % NW) * STRIDE + e / NW] = ex;
        ex += v[i];
    }
    lds_barrier();
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
// step > 1: the minimum and maximum of every step-th element only (a sample).
template <typename K>
__global__ __launch_bounds__(256) void k_probe(const K* __restrict__ a, uint64_t na,
                                               const K* __restrict__ b, uint64_t nb,
                                               uint64_t* __restrict__ minmax, uint64_t step)
{
    __shared__ uint64_t smin[4], smax[4];
    uint64_t mn = ~0ull, mx = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    // U loads in flight per thread; a clamped index re-reads a real element,
    // which leaves the minimum and maximum unchanged.
    constexpr int U = 8;
    const uint64_t sa = (na + step - 1) / step, sb = (nb + step - 1) / step;  // sampled elements
    for (uint64_t i0 = t0; i0 < sa; i0 += stride * U) {
        K v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = ld_clamp(a, (i0 + u * stride) * step, na);
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t o = ord_of(v[u]);
            mn = o < mn ? o : mn;
            mx = o > mx ? o : mx;
        }
    }
    for (uint64_t i0 = t0; i0 < sb; i0 += stride * U) {
        K v[U];
#pragma unroll
        for (int u = 0; u < U; u++) v[u] = ld_clamp(b, (i0 + u * stride) * step, nb);
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint64_t o = ord_of(v[u]);
            mn = o < mn ? o : mn;
            mx = o > mx ? o : mx;
        }
    }
    mn = wave_min64(mn);
    mx = wave_max64(mx);
    if ((threadIdx.x & 63) == 0) {
        smin[threadIdx.x / 64] = mn;
        smax[threadIdx.x / 64] = mx;
    }
    lds_barrier();
    if (threadIdx.x == 0) {
        for (int i = 0; i < 4; i++) {
            mn = smin[i] < mn ? smin[i] : mn;
            mx = smax[i] > mx ? smax[i] : mx;
        }
        atomicMin((unsigned long long*)&minmax[0], (unsigned long long)mn);
        atomicMax((unsigned long long*)&minmax[1], (unsigned long long)mx);
    }
}

hipError_t launch_probe_step(int key_bytes, const void* a, uint64_t na, const void* b, uint64_t nb,
                             uint64_t step, uint64_t* minmax, hipStream_t st)
{
    hipError_t e = launch_fill_u64(minmax, 1, ~0ull, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u64(minmax + 1, 1, 0ull, st);
    if (e != hipSuccess) return e;
    if (step < 1) step = 1;
    const uint64_t n = ((na > nb ? na : nb) + step - 1) / step;
    uint64_t blocks = (n + 256 * 16 - 1) / (256 * 16);
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_probe<int32_t>, dim3((uint32_t)blocks), dim3(256), 0, st,
                           (const int32_t*)a, na, (const int32_t*)b, nb, minmax, step);
    else
        hipLaunchKernelGGL(k_probe<int64_t>, dim3((uint32_t)blocks), dim3(256), 0, st,
                           (const int64_t*)a, na, (const int64_t*)b, nb, minmax, step);
    return hipGetLastError();
}

hipError_t launch_probe(int key_bytes, const void* a, uint64_t na, const void* b, uint64_t nb,
                        uint64_t* minmax, hipStream_t st)
{
    return launch_probe_step(key_bytes, a, na, b, nb, 1, minmax, st);
}

// Every step-th key of a column, as its ordinal: out[i] = ord(a[i * step]) for
// i < ceil(n / step).
template <typename K>
__global__ __launch_bounds__(256) void k_gather_step(const K* __restrict__ a, uint64_t n, uint64_t step,
                                                     uint64_t* __restrict__ out)
{
    const uint64_t m = (n + step - 1) / step;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < m; i += (uint64_t)gridDim.x * 256) out[i] = ord_of(a[i * step]);
}

hipError_t launch_gather_step(int key_bytes, const void* a, uint64_t n, uint64_t step, uint64_t* out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    if (step < 1) step = 1;
    const uint64_t m = (n + step - 1) / step;
    uint64_t blocks = (m + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_gather_step<int32_t>, dim3((uint32_t)blocks), dim3(256), 0, st, (const int32_t*)a, n,
                           step, out);
    else
        hipLaunchKernelGGL(k_gather_step<int64_t>, dim3((uint32_t)blocks), dim3(256), 0, st, (const int64_t*)a, n,
                           step, out);
    return hipGetLastError();
}

// Ordinals of single keys anywhere in the buffers: out[i] = ord of the key at
// refs[i] (4 or 8 bytes). Used to sample a few rows of crowded buckets.
__global__ __launch_bounds__(256) void k_read_ords(const KeyRef* __restrict__ refs, uint32_t n,
                                                   uint64_t* __restrict__ out)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const KeyRef r = refs[i];
    out[i] = r.kb == 8 ? ord_of(*(const int64_t*)r.p) : ord_of(*(const int32_t*)r.p);
}

hipError_t launch_read_ords(const KeyRef* refs, uint32_t n, uint64_t* out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_read_ords, dim3((n + 255) / 256), dim3(256), 0, st, refs, n, out);
    return hipGetLastError();
}

// Digit of ordinal o in a group: its radix digit, or in a pivot group
// (GROUP_PIVOT) its side of the pivot key `base`: 0 below, 1 equal, 2 above.
__device__ __forceinline__ uint32_t group_digit(uint64_t o, uint64_t base, uint32_t shift, uint32_t mask,
                                                bool pivot)
{
    return pivot ? (uint32_t)(o >= base) + (uint32_t)(o > base) : (uint32_t)((o - base) >> shift) & mask;
}

// ---------------------------------------------------------------------------
// radix histogram: per chunk, the digit counts of its rows (and, per group
// and digit, the smallest and largest ordinal, so that every child bucket
// knows its exact key range and single-key buckets are recognised)
// ---------------------------------------------------------------------------
// LEARNED: the digit is the learned bucket of the row's key (model copied to
// LDS), and every row's bucket is stored in bkt for the scatter. The learned
// variant runs 1024-thread blocks: its 34 KiB of LDS per block would cap
// 256-thread blocks at half the waves a CU can hold.
template <typename K, bool LEARNED, int NT = PART_THREADS>
__global__ __launch_bounds__(NT) void k_hist(const ChunkDesc* __restrict__ chunks,
                                                       const GroupDesc* __restrict__ groups,
                                                       BufSet bufs, uint32_t* __restrict__ hist,
                                                       uint64_t* __restrict__ gmin,
                                                       uint64_t* __restrict__ gmax,
                                                       const tj_rmi_t* __restrict__ model, BktSet bkt,
                                                       uint32_t* __restrict__ range_miss)
{
    __shared__ uint32_t cnt[NB];
    __shared__ uint64_t mn[NB], mx[NB];
    __shared__ __align__(16) char lm_raw[LEARNED ? sizeof(tj_rmi_t) : 16];
    const tj_rmi_t& lm = *(const tj_rmi_t*)lm_raw;
    const ChunkDesc ch = chunks[blockIdx.x];
    const GroupDesc g = groups[ch.group];
    const K* __restrict__ src = (const K*)bufs.key[g.src][g.side] + g.src_koff + ch.start;
    uint16_t* __restrict__ bk = LEARNED ? bkt.b[g.side] + ch.start : nullptr;
    const uint32_t nbins = 1u << g.bits;
    for (uint32_t d = threadIdx.x; d < nbins; d += NT) {
        cnt[d] = 0;
        mn[d] = ~0ull;
        mx[d] = 0;
    }
    if (LEARNED) rmi_to_lds<NT>((tj_rmi_t*)lm_raw, model);
    lds_barrier();
    // GROUP_CHECK_RANGE: the digit range came from a sample; a row outside
    // [base, base + nbins << shift) would take a wrong digit, so it is flagged
    // (the planner then probes the exact range and repeats the pass).
    const bool check = !LEARNED && (g.flags & GROUP_CHECK_RANGE) != 0;
    const bool pivot = (g.flags & GROUP_PIVOT) != 0;
    bool miss = false;
    // Rows are counted with LDS atomics. When every valid row of a wave's round
    // falls in one bin (skewed inputs: buckets dominated by one key), the wave
    // reduces them first and one lane updates the bin.
    constexpr int U = 4;
    const uint32_t lane = threadIdx.x & 63;
    for (uint32_t b0 = 0; b0 < ch.len; b0 += NT * U) {  // trip count uniform over the block
        const uint32_t q0 = b0 + threadIdx.x;
        K k[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t q = q0 + u * NT;
            k[u] = ld_clamp(src, q, ch.len);  // rows past the chunk are masked below
        }
        // learned buckets of the round's rows first: independent chains of LDS
        // reads that the compiler interleaves
        uint32_t lb[LEARNED ? U : 1];
        if (LEARNED) {
#pragma unroll
            for (int u = 0; u < U; u++) lb[LEARNED ? u : 0] = min(rmi_bucket(lm, ord_of(k[u])), nbins - 1u);
#pragma unroll
            for (int u = 0; u < U; u++) {
                const uint32_t q = q0 + u * NT;
                if (q < ch.len) bk[q] = (uint16_t)lb[LEARNED ? u : 0];
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const uint32_t q = q0 + u * NT;
            const uint64_t o = ord_of(k[u]);
            const bool valid = q < ch.len && o >= g.flo && o <= g.fhi;
            uint32_t d;
            if (LEARNED) d = valid ? lb[LEARNED ? u : 0] : 0u;
            else d = valid ? group_digit(o, g.base, g.shift, nbins - 1u, pivot) : 0u;
            if (check) miss = miss || (valid && (o < g.base || ((o - g.base) >> g.shift) >= nbins));
            const uint64_t vm = ballot(valid);
            if (vm == 0) continue;
            const int first = __ffsll((unsigned long long)vm) - 1;
            const uint32_t d0 = (uint32_t)__shfl((int)d, first, 64);
            if (ballot(valid && d != d0) == 0) {
                const uint64_t lo = wave_min64(valid ? o : ~0ull);
                const uint64_t hi = wave_max64(valid ? o : 0ull);
                if ((int)lane == first) {
                    atomicAdd(&cnt[d0], (uint32_t)__popcll(vm));
                    atomicMin((unsigned long long*)&mn[d0], (unsigned long long)lo);
                    atomicMax((unsigned long long*)&mx[d0], (unsigned long long)hi);
                }
            } else if (valid) {
                atomicAdd(&cnt[d], 1u);
                // The minimum only falls and the maximum only rises, so a row
                // that does not beat a value read (atomically) at any moment
                // cannot change them; most rows skip the 64-bit atomics.
                if (o < __hip_atomic_load(&mn[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                    atomicMin((unsigned long long*)&mn[d], (unsigned long long)o);
                if (o > __hip_atomic_load(&mx[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
                    atomicMax((unsigned long long*)&mx[d], (unsigned long long)o);
            }
        }
    }
    if (check && ballot(miss) && (threadIdx.x & 63) == 0) atomicOr(range_miss, 1u);
    lds_barrier();
    for (uint32_t d = threadIdx.x; d < nbins; d += NT) {
        hist[(uint64_t)blockIdx.x * NB + d] = cnt[d];
        if (cnt[d]) {
            atomicMin((unsigned long long*)&gmin[g.child0 + d], (unsigned long long)mn[d]);
            atomicMax((unsigned long long*)&gmax[g.child0 + d], (unsigned long long)mx[d]);
        }
    }
}

hipError_t launch_hist(int key_bytes, const ChunkDesc* chunks, uint32_t nchunks,
                       const GroupDesc* groups, BufSet bufs, uint32_t* hist, uint64_t* gmin,
                       uint64_t* gmax, uint32_t* range_miss, hipStream_t st)
{
    if (nchunks == 0) return hipSuccess;
    const BktSet none{};
    if (key_bytes == 4)
        hipLaunchKernelGGL((k_hist<int32_t, false>), dim3(nchunks), dim3(PART_THREADS), 0, st, chunks, groups,
                           bufs, hist, gmin, gmax, nullptr, none, range_miss);
    else
        hipLaunchKernelGGL((k_hist<int64_t, false>), dim3(nchunks), dim3(PART_THREADS), 0, st, chunks, groups,
                           bufs, hist, gmin, gmax, nullptr, none, range_miss);
    return hipGetLastError();
}

constexpr int LEARNED_HIST_THREADS = 1024;

hipError_t launch_learned_hist(int key_bytes, const ChunkDesc* chunks, uint32_t nchunks,
                               const GroupDesc* groups, BufSet bufs, const tj_rmi_t* model, BktSet bkt,
                               uint32_t* hist, uint64_t* gmin, uint64_t* gmax, hipStream_t st)
{
    if (nchunks == 0) return hipSuccess;
    if (key_bytes == 4)
        hipLaunchKernelGGL((k_hist<int32_t, true, LEARNED_HIST_THREADS>), dim3(nchunks), dim3(LEARNED_HIST_THREADS), 0, st,
                           chunks, groups,
                           bufs, hist, gmin, gmax, model, bkt, nullptr);
    else
        hipLaunchKernelGGL((k_hist<int64_t, true, LEARNED_HIST_THREADS>), dim3(nchunks), dim3(LEARNED_HIST_THREADS), 0, st,
                           chunks, groups,
                           bufs, hist, gmin, gmax, model, bkt, nullptr);
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

// one block per segment, one thread per digit
__global__ __launch_bounds__(NB) void k_children(const GroupDesc* __restrict__ groups, int nside,
                                                 const uint32_t* __restrict__ ccount,
                                                 const uint64_t* __restrict__ gmin,
                                                 const uint64_t* __restrict__ gmax,
                                                 ChildRec* __restrict__ out)
{
    const GroupDesc g0 = groups[blockIdx.x * nside];
    const uint32_t d = threadIdx.x;
    if (d >= (1u << g0.bits)) return;
    ChildRec c;
    c.rn = ccount[g0.child0 + d];
    c.lo = gmin[g0.child0 + d];
    c.hi = gmax[g0.child0 + d];
    c.sn = 0;
    if (nside == 2) {
        const uint32_t c1 = groups[blockIdx.x * 2 + 1].child0 + d;
        c.sn = ccount[c1];
        c.lo = gmin[c1] < c.lo ? gmin[c1] : c.lo;
        c.hi = gmax[c1] > c.hi ? gmax[c1] : c.hi;
    }
    out[g0.child0 / nside + d] = c;
}

hipError_t launch_children(const GroupDesc* groups, uint32_t ngroups, int nside,
                           const uint32_t* ccount, const uint64_t* gmin, const uint64_t* gmax,
                           ChildRec* out, hipStream_t st)
{
    if (ngroups == 0) return hipSuccess;
    hipLaunchKernelGGL(k_children, dim3(ngroups / nside), dim3(NB), 0, st, groups, nside, ccount, gmin,
                       gmax, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Leaf batching of a level on the device, for levels of many segments whose
// children mostly fit one LDS block: the host then reads back four summary
// words and the few children too large for a leaf instead of one record per
// child. One wave per segment. Adjacent children are batched
// greedily into leaves of at most LEAF_CAP rows (a child whose keys were
// narrowed into another 2^32 window starts a new leaf), as the host planner
// does. A child over LEAF_CAP closes the open leaf and is listed for the host
// (BigChild records at the top of the leaf table, counted in summary[4]): the
// host plans only those. The greedy choice is the only sequential part: a
// uniform loop over the children's row counts marks where leaves start (a
// 512-bit mask in scalar registers). Everything else is per child, across the
// lanes: exclusive prefix sums of the rows give each leaf its first rows and
// sizes, the last non-empty child before the leaf's end gives its largest key,
// and a prefix count of children with rows on both sides tells whether a join
// leaf can produce pairs. Pass 0 counts the useful leaves and the listed
// children of each segment; pass 1 writes them after those of the earlier
// segments of the batch (leaves upwards from leaf_base, listed children
// downwards from the top of the table; a slot below leaf_base sets
// BATCH_OVERFLOW, and so does a collision, which the host detects from the
// totals).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_batch_leaves(const GroupDesc* __restrict__ groups,
                                                     const ChildRec* __restrict__ crec, BatchArgs a,
                                                     uint32_t* __restrict__ seg_count,
                                                     LeafDesc* __restrict__ leaves,
                                                     unsigned long long* __restrict__ summary, int pass)
{
    constexpr int RPL = NB / 64;  // children per lane: child d = j*64 + lane
    __shared__ uint32_t s_rpre[NB + 1], s_spre[NB + 1], s_both[NB + 1];  // exclusive prefixes
    __shared__ uint32_t s_last[NB];  // last non-empty child at or before d
    __shared__ uint64_t s_hi[NB];
    const uint32_t sgi = blockIdx.x, l = threadIdx.x;
    const GroupDesc g0 = groups[sgi * a.nside];
    const uint64_t s_start = a.nside == 2 ? groups[sgi * 2 + 1].dst_start : 0;
    const uint64_t koff_s = a.nside == 2 ? groups[sgi * 2 + 1].dst_koff : 0;
    const uint32_t nb = 1u << g0.bits;
    const ChildRec* cr = crec + g0.child0 / a.nside;
    uint32_t rows[RPL], win[RPL];
    uint64_t lo[RPL];
    uint64_t bigm[RPL];  // children over LEAF_CAP, one bit each
    uint32_t rc = 0, sc = 0, bc = 0, lastc = 0;  // carries of the prefixes across slots
#pragma unroll
    for (int j = 0; j < RPL; j++) {
        const uint32_t d = j * 64 + l;
        const ChildRec c = d < nb ? cr[d] : ChildRec{0, 0, ~0ull, 0};
        rows[j] = c.rn + c.sn;
        bigm[j] = ballot(rows[j] > (uint32_t)LEAF_CAP);
        uint64_t clo = c.lo, chi = c.hi;
        win[j] = 0;
        if (a.narrowing && rows[j]) {
            const uint64_t off = clo - g0.base;
            win[j] = (uint32_t)(off >> 32);
            clo = off & 0xffffffffull;
            chi = (chi - g0.base) & 0xffffffffull;
        }
        lo[j] = clo;
        const uint32_t both = c.rn > 0 && c.sn > 0 ? 1u : 0u;
        const uint32_t ri = wave_incl_scan(c.rn), si = wave_incl_scan(c.sn), bi = wave_incl_scan(both);
        const uint32_t li = wave_incl_max(rows[j] ? d + 1 : 0u);  // 1 + last non-empty child so far
        if (d < nb) {
            s_rpre[d] = rc + ri - c.rn;
            s_spre[d] = sc + si - c.sn;
            s_both[d] = bc + bi - both;
            const uint32_t lst = li > lastc ? li : lastc;
            s_last[d] = lst ? lst - 1 : 0u;
            s_hi[d] = chi;
        }
        rc += (uint32_t)__shfl((int)ri, 63, 64);
        sc += (uint32_t)__shfl((int)si, 63, 64);
        bc += (uint32_t)__shfl((int)bi, 63, 64);
        const uint32_t lm = (uint32_t)__shfl((int)li, 63, 64);
        lastc = lm > lastc ? lm : lastc;
    }
    if (l == 0) {
        s_rpre[nb] = rc;
        s_spre[nb] = sc;
        s_both[nb] = bc;
    }
    // greedy batching: bit d of start[] marks a child that opens a leaf
    uint64_t start[RPL];
    {
        bool open = false;
        uint32_t acc = 0, lwin = 0;
#pragma unroll
        for (int j = 0; j < RPL; j++) {
            uint64_t m = 0;
            const uint64_t ne = ballot(rows[j] > 0);
            uint64_t todo = ne;
            while (todo) {
                const uint32_t ln = (uint32_t)__builtin_ctzll(todo);
                todo &= todo - 1;
                const uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)rows[j], (int)ln);
                if (r > (uint32_t)LEAF_CAP) {  // listed for the host; the next child opens a leaf
                    open = false;
                    continue;
                }
                const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)win[j], (int)ln);
                if (!open || w != lwin || acc + r > (uint32_t)LEAF_CAP) {
                    m |= 1ull << ln;
                    open = true;
                    lwin = w;
                    acc = 0;
                }
                acc += r;
            }
            start[j] = m;
        }
    }
    lds_barrier();  // the prefix tables are complete
    // per leaf (its starting child): extent, sizes, key range, usefulness
    uint32_t useful[RPL], e_of[RPL];
#pragma unroll
    for (int j = 0; j < RPL; j++) {
        const uint32_t d = j * 64 + l;
        const bool st = (start[j] >> l) & 1ull;
        // the leaf ends at the next start or listed child after d, else at
        // the end of the segment's children
        uint32_t e = nb;
        const uint64_t above = l == 63 ? 0ull : (start[j] | bigm[j]) & (~0ull << (l + 1));
        if (above) {
            e = j * 64 + (uint32_t)__builtin_ctzll(above);
        } else {
#pragma unroll
            for (int k = j + 1; k < RPL; k++)
                if (e == nb && (start[k] | bigm[k])) e = k * 64 + (uint32_t)__builtin_ctzll(start[k] | bigm[k]);
        }
        e_of[j] = e;
        useful[j] = st && (!a.join || s_both[e] - s_both[d] > 0) ? 1u : 0u;
    }
    // emission order: useful leaves, and listed children, in child order
    uint32_t idx[RPL], bidx[RPL], nleaf = 0, nbig = 0;
#pragma unroll
    for (int j = 0; j < RPL; j++) {
        const uint64_t um = ballot(useful[j] != 0);
        idx[j] = nleaf + mbcnt(um);
        nleaf += (uint32_t)__popcll(um);
        bidx[j] = nbig + mbcnt(bigm[j]);
        nbig += (uint32_t)__popcll(bigm[j]);
    }
    if (pass == 0) {
        if (l == 0) seg_count[sgi] = nleaf | (nbig << 16);
        return;
    }
    uint64_t before = 0, before_big = 0;
    for (uint32_t i = l; i < sgi; i += 64) {
        before += seg_count[i] & 0xffffu;
        before_big += seg_count[i] >> 16;
    }
    before = wave_sum64(before);
    before_big = wave_sum64(before_big);
    uint64_t rows_all = 0;
    bool wide = false, over = false;
#pragma unroll
    for (int j = 0; j < RPL; j++) {
        if (!((bigm[j] >> l) & 1ull)) continue;
        const uint32_t d = j * 64 + l;
        const uint64_t k = before_big + bidx[j];
        if (a.leaf_base + k + 1 > a.leaf_cap) {
            over = true;
            continue;
        }
        const ChildRec c = cr[d];
        BigChild b;
        b.seg = sgi;
        b.child = d;
        b.r_off = s_rpre[d];
        b.s_off = s_spre[d];
        b.rn = c.rn;
        b.sn = c.sn;
        b.lo = c.lo;
        b.hi = c.hi;
        *(BigChild*)(leaves + (a.leaf_cap - 1 - k)) = b;
    }
#pragma unroll
    for (int j = 0; j < RPL; j++) {
        if (!useful[j]) continue;
        const uint32_t d = j * 64 + l, e = e_of[j];
        const uint32_t rn = s_rpre[e] - s_rpre[d], sn = s_spre[e] - s_spre[d];
        rows_all += (uint64_t)rn + sn;
        const uint64_t slot = a.leaf_base + before + idx[j];
        if (slot >= a.leaf_cap) {
            over = true;
            continue;
        }
        const uint64_t llo = lo[j], lhi = s_hi[s_last[e - 1]];
        const uint64_t span = lhi - llo;
        const uint32_t bits = span ? 64u - (uint32_t)__clzll((long long)span) : 0u;
        wide = wide || bits > 32;
        LeafDesc L;
        L.r0 = g0.dst_start + s_rpre[d];
        L.s0 = s_start + s_spre[d];
        L.kr0 = L.r0 + g0.dst_koff;
        L.ks0 = L.s0 + koff_s;
        L.base = llo;
        L.out = a.join ? 0 : L.r0 + a.out_delta;
        L.rn = rn;
        L.sn = sn;
        L.bits = (uint16_t)bits;
        L.kb = (uint16_t)a.kb;
        L.buf = (uint16_t)a.buf;
        L.flags = (uint16_t)a.flags;
        leaves[slot] = L;
    }
    rows_all = wave_sum64(rows_all);
    const uint64_t fl = (ballot(wide) ? BATCH_WIDE : 0ull) | (ballot(over) ? BATCH_OVERFLOW : 0ull);
    if (l != 0) return;
    atomicAdd(&summary[0], (unsigned long long)nleaf);
    atomicAdd(&summary[1], (unsigned long long)rows_all);
    if (fl) atomicOr(&summary[2], (unsigned long long)fl);
    if (nbig) atomicAdd(&summary[4], (unsigned long long)nbig);
}

hipError_t launch_batch_leaves(const GroupDesc* groups, const ChildRec* crec, const BatchArgs& a,
                               uint32_t* seg_count, LeafDesc* leaves, uint64_t* summary, int pass,
                               hipStream_t st)
{
    if (a.nseg == 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_leaves, dim3(a.nseg), dim3(64), 0, st, groups, crec, a, seg_count, leaves,
                       (unsigned long long*)summary, pass);
    return hipGetLastError();
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
// SC_TILE rows. Per tile: rows are ranked within their wave by ballot match,
// offset across waves and digits by one block scan, staged in LDS grouped by
// digit, and written out as per-digit runs while the next tile's loads are in
// flight. Wave w of the tile owns rows [w*SC_KI*64, (w+1)*SC_KI*64); round r
// of a wave covers 64 consecutive rows, so (wave, round, lane) is input order
// and the partition is stable.
// KO is the written key type. KO = int32 with K = int64 narrows the keys: a
// row is written as the low 32 bits of (ord - g.base), stored so that ord_of
// of the stored int32 gives them back. Every child of such a pass spans at
// most 2^32 ordinals and lies inside one window g.base + [j*2^32, (j+1)*2^32),
// so inside a child (and among children of one window) the narrowed keys
// order as the originals.
// ---------------------------------------------------------------------------
constexpr int SC_NT = 512, SC_KI = 18, SC_NW = SC_NT / 64, SC_TILE = SC_NT * SC_KI;
constexpr int SC_STRIDE = NB + 1;
static_assert(SC_TILE == PART_TILE, "chunk sizes are planned in scatter tiles");

// DIGIN (learned pass): each row's digit is read from bkt instead of being
// computed from its key; rows are ranked by ballot match, which is stable by
// construction, and the staged digit replaces the staged tile index.
template <typename K, typename KO, bool RIDS, bool WKEYS, bool DIGIN>
__global__ __launch_bounds__(SC_NT) void k_scatter(const ChunkDesc* __restrict__ chunks,
                                                   const GroupDesc* __restrict__ groups,
                                                   const uint32_t* __restrict__ hist,
                                                   const uint32_t* __restrict__ cbsum,
                                                   const uint64_t* __restrict__ cstart,
                                                   BufSet bufs, BktSet bkt)
{
    constexpr int NT = SC_NT, KI = SC_KI, NW = SC_NW, TILE = SC_TILE;
    __shared__ uint32_t cnt[NW * SC_STRIDE];
    __shared__ uint32_t spare[NT];  // one private counter per thread for rows that take no part
    __shared__ uint32_t run[NB], delta[NB];
    __shared__ uint32_t tmp[NW];
    __shared__ uint32_t s_unordered;
    // staging, with one spare slot per lane of a wave for rows that take no part
    __shared__ K skey[TILE + 64];
    __shared__ int32_t srid[RIDS ? TILE + 64 : 1];
    __shared__ uint16_t sidx[TILE + 64];  // the staged row's index inside the tile (DIGIN: its digit)

    const ChunkDesc ch = chunks[blockIdx.x];
    const GroupDesc g = groups[ch.group];
    const K* __restrict__ src_k = (const K*)bufs.key[g.src][g.side] + g.src_koff + ch.start;
    const int32_t* __restrict__ src_r = bufs.rid[g.src][g.side] + ch.start;
    KO* __restrict__ dst_k = (KO*)bufs.key[g.dst][g.side] + g.dst_koff;
    int32_t* __restrict__ dst_r = (int32_t*)bufs.rid[g.dst][g.side];
    const uint16_t* __restrict__ src_b = DIGIN ? bkt.b[g.side] + ch.start : nullptr;
    const uint32_t nbins = 1u << g.bits, mask = nbins - 1u;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    const bool force_reorder = (g.flags & GROUP_FORCE_REORDER) != 0;

    const bool pivot = (g.flags & GROUP_PIVOT) != 0;
    auto digit_of = [&](K k) { return group_digit(ord_of(k), g.base, g.shift, mask, pivot); };
    // a narrowing launch may hold groups that keep their 8-byte keys (uniform per block)
    const bool wide = sizeof(KO) < sizeof(K) && (g.flags & GROUP_WIDE) != 0;
    K* __restrict__ dst_kw = (K*)bufs.key[g.dst][g.side] + g.dst_koff;
    auto write_row = [&](uint32_t dst, K k, int32_t rid) {
        if (WKEYS) {
            if (sizeof(KO) == sizeof(K)) dst_k[dst] = (KO)k;
            else if (wide) dst_kw[dst] = k;
            else dst_k[dst] = (KO)((uint32_t)(ord_of(k) - g.base) ^ 0x80000000u);
        }
        if (RIDS) dst_r[dst] = rid;
    };

    for (uint32_t d = threadIdx.x; d < NB; d += NT)
        run[d] = d < nbins ? (uint32_t)(cstart[g.child0 + d] + cbsum[(uint64_t)ch.cblock * NB + d] +
                                        hist[(uint64_t)blockIdx.x * NB + d])
                           : 0u;
    K key[KI];
    int32_t rid[KI];
    uint32_t bin[DIGIN ? KI : 1];
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        key[r] = q < ch.len ? src_k[q] : K(0);
        if (RIDS) rid[r] = q < ch.len ? src_r[q] : 0;
        if (DIGIN) bin[DIGIN ? r : 0] = ld_clamp(src_b, q, ch.len);  // rows past the chunk are masked
    }
    for (uint32_t t0 = 0; t0 < ch.len; t0 += TILE) {
        uint32_t dig[KI], rk[KI];
        bool val[KI];
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = t0 + (w * KI + r) * 64 + l;
            const uint64_t o = ord_of(key[r]);
            val[r] = q < ch.len && o >= g.flo && o <= g.fhi;
            if (DIGIN) dig[r] = val[r] ? bin[DIGIN ? r : 0] & mask : 0u;
            else dig[r] = val[r] ? group_digit(o, g.base, g.shift, mask, pivot) : 0u;
        }
        for (uint32_t i = l; i < NB; i += 64) cnt[w * SC_STRIDE + i] = 0;
        // Rank inside the wave: one LDS atomic per row on the wave's own
        // counters. The wave issues its rounds in row order; within a round the
        // hardware applies the lanes that hit one counter in lane order, which
        // makes the ranks stable. Nothing relies on that order: the write-out
        // checks it and the tile is written again, ranked by ballots, if a
        // digit's rows ever come out of input order.
        if (DIGIN) {
#pragma unroll
            for (int r = 0; r < KI; r++) rk[r] = wave_rank(dig[r], val[r], (int)g.bits, &cnt[w * SC_STRIDE]);
        } else {
#pragma unroll
            for (int r = 0; r < KI; r++)
                rk[r] = atomicAdd(val[r] ? &cnt[w * SC_STRIDE + dig[r]] : &spare[threadIdx.x], 1u);
        }
        if (threadIdx.x == 0) s_unordered = 0;
        lds_barrier();
        const uint32_t total = scan_counts<NT, NW, NB>(cnt, tmp);
        for (uint32_t d = threadIdx.x; d < NB; d += NT) {
            const uint32_t tex = cnt[d];
            const uint32_t nxt = d + 1 < NB ? cnt[d + 1] : total;
            delta[d] = run[d] - tex;
            run[d] += nxt - tex;
        }
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t p = val[r] ? cnt[w * SC_STRIDE + dig[r]] + rk[r] : TILE + l;
            skey[p] = key[r];
            if (RIDS) srid[p] = rid[r];
            sidx[p] = (uint16_t)(DIGIN ? dig[r] : (w * KI + r) * 64 + l);
        }
        lds_barrier();
        // next tile's loads overlap the write-out of this one
        const uint32_t n0 = t0 + TILE;
        if (n0 < ch.len) {
#pragma unroll
            for (int r = 0; r < KI; r++) {
                const uint32_t q = n0 + (w * KI + r) * 64 + l;
                key[r] = q < ch.len ? src_k[q] : K(0);
                if (RIDS) rid[r] = q < ch.len ? src_r[q] : 0;
                if (DIGIN) bin[DIGIN ? r : 0] = ld_clamp(src_b, q, ch.len);
            }
        }
        bool unordered = false;
        if (total) {
            // the KI rows of each thread are read together (a position past the
            // tile's rows re-reads its last row and writes nothing)
#pragma unroll
            for (int j = 0; j < KI; j++) {
                const uint32_t p = threadIdx.x + j * NT;
                const uint32_t pc = p < total ? p : total - 1;
                const K k = skey[pc];
                const int32_t rv = RIDS ? srid[pc] : 0;
                const uint32_t x = sidx[pc], xp = DIGIN ? 0u : sidx[pc ? pc - 1 : 0];
                const uint32_t d = DIGIN ? x : digit_of(k);
                if (p < total) {
                    write_row(delta[d] + p, k, rv);
                    // cnt[d] (wave 0's entry) is where digit d starts inside the tile
                    if (!DIGIN) unordered = unordered || (p > cnt[d] && xp > x);
                }
            }
        }
        if (unordered) s_unordered = 1;
        lds_barrier();
        if (!DIGIN && (s_unordered || force_reorder)) {
            // Rare path: rank the tile again by ballot match (from its rows in
            // the source) and write it over the same destination rows.
            K k2[KI];
            int32_t r2[KI];
#pragma unroll
            for (int r = 0; r < KI; r++) {
                const uint32_t q = t0 + (w * KI + r) * 64 + l;
                k2[r] = q < ch.len ? src_k[q] : K(0);
                r2[r] = RIDS && q < ch.len ? src_r[q] : 0;
                const uint64_t o = ord_of(k2[r]);
                val[r] = q < ch.len && o >= g.flo && o <= g.fhi;
                dig[r] = val[r] ? group_digit(o, g.base, g.shift, mask, pivot) : 0u;
            }
            for (uint32_t i = l; i < NB; i += 64) cnt[w * SC_STRIDE + i] = 0;
#pragma unroll
            for (int r = 0; r < KI; r++) rk[r] = wave_rank(dig[r], val[r], (int)g.bits, &cnt[w * SC_STRIDE]);
            lds_barrier();
            scan_counts<NT, NW, NB>(cnt, tmp);  // same counts, so delta[] still holds
#pragma unroll
            for (int r = 0; r < KI; r++) {
                if (val[r]) {
                    const uint32_t p = cnt[w * SC_STRIDE + dig[r]] + rk[r];
                    skey[p] = k2[r];
                    if (RIDS) srid[p] = r2[r];
                }
            }
            lds_barrier();
            for (uint32_t p = threadIdx.x; p < total; p += NT) {
                const K k = skey[p];
                write_row(delta[digit_of(k)] + p, k, RIDS ? srid[p] : 0);
            }
            lds_barrier();
        }
    }
}

hipError_t launch_scatter(int key_bytes, int out_key_bytes, bool rids, bool keys, const ChunkDesc* chunks,
                          uint32_t nchunks, const GroupDesc* groups, const uint32_t* hist,
                          const uint32_t* cbsum, const uint64_t* cstart, BufSet bufs, hipStream_t st)
{
    if (nchunks == 0) return hipSuccess;
    if (out_key_bytes > key_bytes) return hipErrorInvalidValue;
    const dim3 grid(nchunks), block(SC_NT);
    const BktSet none{};
#define TJ_SC(K, KO, R, W)                                                                           \
    hipLaunchKernelGGL((k_scatter<K, KO, R, W, false>), grid, block, 0, st, chunks, groups, hist, cbsum, cstart, \
                       bufs, none)
    if (key_bytes == 4) {
        if (!keys) TJ_SC(int32_t, int32_t, true, false);
        else if (rids) TJ_SC(int32_t, int32_t, true, true);
        else TJ_SC(int32_t, int32_t, false, true);
    } else if (out_key_bytes == 8 || !keys) {
        if (!keys) TJ_SC(int64_t, int64_t, true, false);
        else if (rids) TJ_SC(int64_t, int64_t, true, true);
        else TJ_SC(int64_t, int64_t, false, true);
    } else {
        if (rids) TJ_SC(int64_t, int32_t, true, true);
        else TJ_SC(int64_t, int32_t, false, true);
    }
#undef TJ_SC
    return hipGetLastError();
}

hipError_t launch_learned_scatter(int key_bytes, bool rids, const ChunkDesc* chunks, uint32_t nchunks,
                                  const GroupDesc* groups, const uint32_t* hist, const uint32_t* cbsum,
                                  const uint64_t* cstart, BufSet bufs, BktSet bkt, hipStream_t st)
{
    if (nchunks == 0) return hipSuccess;
    const dim3 grid(nchunks), block(SC_NT);
#define TJ_SCL(K, R)                                                                                  \
    hipLaunchKernelGGL((k_scatter<K, K, R, true, true>), grid, block, 0, st, chunks, groups, hist, cbsum,  \
                       cstart, bufs, bkt)
    if (key_bytes == 4) {
        if (rids) TJ_SCL(int32_t, true);
        else TJ_SCL(int32_t, false);
    } else {
        if (rids) TJ_SCL(int64_t, true);
        else TJ_SCL(int64_t, false);
    }
#undef TJ_SCL
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
constexpr int LBINS = 256, LSTRIDE = LBINS + 1;
// Leaf block shape per key word: 32-bit keys use 512 threads x 16 rows (57 KB
// of LDS, two blocks per CU); 64-bit keys 1024 threads x 8 rows (97 KB, one
// block of 16 waves per CU).
template <typename KW> struct LeafShape {
    static constexpr int NT = sizeof(KW) == 4 ? 512 : 1024;
    static constexpr int KI = LEAF_CAP / NT;
    static constexpr int NW = NT / 64;
    static constexpr int NBB = sizeof(KW) == 4 ? 12 : 13;  // bin bits of block_bin_sort
    static constexpr int NBIN = 1 << NBB;
    // LDS words shared by the bin counters and the LSD digit counters
    static constexpr int CNT_WORDS = NBIN > NW * LSTRIDE ? NBIN : NW * LSTRIDE;
};

// LDS array whose element i sits at i + (i / G) * S: S spare elements after
// every G. With G = the items per thread, a wave reading its items in blocked
// order (lane l at l*G + i) has an odd stride in 4-byte words and so spreads
// its lanes over the banks; consecutive-lane access stays conflict-free.
template <typename T, int G, int S>
struct LdsPad {
    T* p;
    __device__ __forceinline__ T& operator[](uint32_t i) const { return p[i + (i / G) * S]; }
    // element t*G + i, i < G (thread t's i-th item in blocked order)
    __device__ __forceinline__ T& blk(uint32_t t, uint32_t i) const { return p[t * (G + S) + i]; }
    // all G items of thread t; 16-byte loads for an unpadded 16-bit array (a
    // wave then reads 16 bytes per lane instead of 2, with 8x fewer conflicts)
    __device__ __forceinline__ void blk_all(uint32_t t, uint32_t (&out)[G]) const
    {
        if constexpr (S == 0 && sizeof(T) == 2 && (G * 2) % 16 == 0) {
            const uint4* v = (const uint4*)(p + t * G);
#pragma unroll
            for (int j = 0; j < G * 2 / 16; j++) {
                const uint4 w = v[j];
                const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
                for (int h = 0; h < 4; h++) {
                    out[j * 8 + 2 * h] = ws[h] & 0xffffu;
                    out[j * 8 + 2 * h + 1] = ws[h] >> 16;
                }
            }
        } else {
#pragma unroll
            for (int i = 0; i < G; i++) out[i] = p[t * (G + S) + i];
        }
    }
    static constexpr uint32_t size(uint32_t n) { return n + (n / G) * S; }
};
// join blocks read their sorted items in blocked order (padded layout); the
// sort blocks read them across lanes (plain layout)
template <typename KW> using KeyLds = LdsPad<KW, LeafShape<KW>::KI, 1>;
template <typename KW> using IdxLds = LdsPad<uint16_t, LeafShape<KW>::KI, 2>;
template <typename KW> using KeyPlain = LdsPad<KW, LeafShape<KW>::KI, 0>;
template <typename KW> using IdxPlain = LdsPad<uint16_t, LeafShape<KW>::KI, 0>;

// Largest bin block_bin_sort accepts: the exact ranking inside a bin costs
// every item of the bin one pass over it.
constexpr uint32_t BIN_MAXC = 48;  // < 64: the bin size is packed in 6 bits

// Stable sort of the block's items in one counting pass. Item key[r] sits at
// position q = (w*KI + r)*64 + l; items with q < n are sorted, the rest are
// padding and stay at q (their keys are all ones and their positions the
// largest, so that is their sorted place too). An item's index is its
// position q, so the stable order is the order of the pairs (key, q).
//  1. Each item is counted into one of 2^NBB bins by the top bits of its key
//     (LDS atomics; the slot an item gets inside its bin is arbitrary).
//  2. An exclusive scan of the bin counts gives each bin's first position;
//     the items are written there in slot order.
//  3. Each item of a bin with two or more items counts the items of its bin
//     that precede it in (key, q) order and moves to that rank.
// The result, in lds_key / lds_idx, is exact whatever order the atomics take.
// Returns false, having written nothing to lds_key / lds_idx, when some bin
// holds more than BIN_MAXC items; the caller then sorts another way.
template <typename KW, int NT, int KI, int NBB, typename KA, typename IA>
__device__ __forceinline__ bool block_bin_sort(const KW (&key)[KI], int bits, uint32_t n, KA lds_key,
                                               IA lds_idx, uint32_t* hist, uint32_t* tmp)
{
    constexpr int NBIN = 1 << NBB, BPT = NBIN / NT;
    static_assert(NBIN % NT == 0, "bins must split evenly over the block");
    static_assert(NT * KI <= 8192, "positions are packed in 13 bits");
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    const int hb = bits < NBB ? bits : NBB;
    const int sh = bits - hb;
    for (uint32_t i = threadIdx.x; i < (uint32_t)NBIN; i += NT) hist[i] = 0;
    lds_barrier();
    // per item: bin | slot << 16, then pos | first of bin << 13 | bin size << 26,
    // then (1 << 31 | final position) for the items that move
    // (array elements are only ever assigned unconditionally: a conditional
    // assignment makes the compiler copy the whole array through every branch)
    uint32_t info[KI];
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        const KW kb = key[r] >> sh;  // < 2^NBB when the keys span `bits` bits
        const uint32_t b = kb < (KW)NBIN ? (uint32_t)kb : (uint32_t)NBIN - 1u;
        uint32_t slot = 0;
        if (q < n) slot = atomicAdd(&hist[b], 1u);
        info[r] = b | (slot << 16);
    }
    lds_barrier();
    uint32_t c[BPT], sum = 0, mx = 0;
#pragma unroll
    for (int i = 0; i < BPT; i++) {
        c[i] = hist[threadIdx.x * BPT + i];
        sum += c[i];
        mx = c[i] > mx ? c[i] : mx;
    }
    if (block_max<NT>(mx, tmp) > BIN_MAXC) return false;
    uint32_t tot;
    uint32_t ex = block_excl_scan<NT>(sum, tmp, &tot);
#pragma unroll
    for (int i = 0; i < BPT; i++) {
        hist[threadIdx.x * BPT + i] = ex;
        ex += c[i];
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        const uint32_t b = info[r] & 0xffffu;
        const uint32_t s0 = hist[b];
        const uint32_t e0 = b + 1 < (uint32_t)NBIN ? hist[b + 1] : n;
        const bool valid = q < n;
        const uint32_t pos = valid ? s0 + (info[r] >> 16) : q;
        info[r] = valid ? pos | (s0 << 13) | ((e0 - s0) << 26) : 0u;
        lds_key[pos] = key[r];
        lds_idx[pos] = (uint16_t)q;
    }
    lds_barrier();
    // The thread's items walk their bins in step, so that the LDS reads of all
    // of them are in flight together: step j reads element j of each bin (an
    // item whose bin is shorter re-reads its bin's first element and ignores it).
    uint32_t rank[KI], cbmax = 0;
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t cb = info[r] >> 26;
        rank[r] = 0;
        cbmax = cb > 1 && cb > cbmax ? cb : cbmax;
    }
    for (uint32_t j = 0; j < cbmax; j++) {
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = (w * KI + r) * 64 + l;
            const uint32_t s0 = (info[r] >> 13) & 0x1fffu, cb = info[r] >> 26;
            const bool act = j < cb;
            const uint32_t e = act ? s0 + j : s0;
            const KW kj = lds_key[e];
            const uint32_t ij = lds_idx[e];
            rank[r] += (act && (kj < key[r] || (kj == key[r] && ij < q))) ? 1u : 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t pos = info[r] & 0x1fffu, s0 = (info[r] >> 13) & 0x1fffu, cb = info[r] >> 26;
        info[r] = (cb > 1 && s0 + rank[r] != pos) ? 0x80000000u | (s0 + rank[r]) : 0u;
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < KI; r++) {
        if (info[r] >> 31) {
            const uint32_t q = (w * KI + r) * 64 + l;
            lds_key[info[r] & 0x1fffu] = key[r];
            lds_idx[info[r] & 0x1fffu] = (uint16_t)q;
        }
    }
    lds_barrier();
    return true;
}

// ATOMIC ranks with one LDS atomic per item (in lane order on this hardware,
// which makes every pass stable); the caller must then check that the result
// is ordered by (key, idx) and sort again with ATOMIC = false if it is not.
template <typename KW, int NT, int KI, bool ATOMIC = false, typename KA, typename IA>
__device__ __forceinline__ void block_lsd_sort(KW (&key)[KI], uint16_t (&idx)[KI], int bits,
                                               KA lds_key, IA lds_idx, uint32_t* cnt,
                                               uint32_t* tmp, int lo_bit = 0)
{
    constexpr int NW = NT / 64;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    const int passes = (bits + 7) / 8;
    if (passes == 0) {
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = (w * KI + r) * 64 + l;
            lds_key[q] = key[r];
            lds_idx[q] = idx[r];
        }
        lds_barrier();
        return;
    }
    for (int p = 0; p < passes; p++) {
        const int sh = lo_bit + 8 * p;
        const int nb = bits - 8 * p < 8 ? bits - 8 * p : 8;
        const uint32_t mask = (1u << nb) - 1u;
        uint32_t dig[KI], rk[KI];
#pragma unroll
        for (int r = 0; r < KI; r++) dig[r] = (uint32_t)(key[r] >> sh) & mask;
        for (uint32_t i = l; i < LBINS; i += 64) cnt[w * LSTRIDE + i] = 0;
        if (ATOMIC) {
#pragma unroll
            for (int r = 0; r < KI; r++) rk[r] = atomicAdd(&cnt[w * LSTRIDE + dig[r]], 1u);
        } else {
#pragma unroll
            for (int r = 0; r < KI; r++) rk[r] = wave_rank(dig[r], true, nb, &cnt[w * LSTRIDE]);
        }
        lds_barrier();
        scan_counts<NT, NW, LBINS>(cnt, tmp);
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t pos = cnt[w * LSTRIDE + dig[r]] + rk[r];
            lds_key[pos] = key[r];
            lds_idx[pos] = idx[r];
        }
        lds_barrier();
        // (reloaded after the last pass too: a conditional reload would make
        // the compiler copy both arrays through the branch)
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = (w * KI + r) * 64 + l;
            key[r] = lds_key[q];
            idx[r] = lds_idx[q];
        }
    }
}

// True (the same on every thread) when the first n items of lds_key/lds_idx
// are in strictly increasing (key, idx) order. *flag must be 0 on entry and
// is 0 again on return; ends with a barrier.
template <typename KW, int NT, int KI, typename KA, typename IA>
__device__ __forceinline__ bool block_check_order(KA lds_key, IA lds_idx, uint32_t n, uint32_t* flag)
{
    const uint32_t t = threadIdx.x, p0 = t * KI;
    KW kp = t ? lds_key.blk(t - 1, KI - 1) : (KW)0;
    uint32_t ip = t ? lds_idx.blk(t - 1, KI - 1) : 0u;
    uint32_t xs[KI];
    lds_idx.blk_all(t, xs);
    bool bad = false;
#pragma unroll
    for (int i = 0; i < KI; i++) {
        const uint32_t p = p0 + i;
        const KW k = lds_key.blk(t, i);
        const uint32_t x = xs[i];
        bad = bad || (p > 0 && p < n && !(kp < k || (kp == k && ip < x)));
        kp = k;
        ip = x;
    }
    if (bad) *flag = 1;
    lds_barrier();
    const bool ok = *flag == 0;
    lds_barrier();
    if (threadIdx.x == 0) *flag = 0;
    return ok;
}

template <typename K, typename KW>
__global__ __launch_bounds__(LeafShape<KW>::NT)
__attribute__((amdgpu_waves_per_eu(4))) void k_leaf_sort(const LeafDesc* __restrict__ leaves,
                                                            BufSet bufs, K* __restrict__ out_k,
                                                            int32_t* __restrict__ out_r)
{
    constexpr int NT = LeafShape<KW>::NT, KI = LeafShape<KW>::KI, NW = LeafShape<KW>::NW, C = LEAF_CAP;
    __shared__ KW lds_key_raw[C];
    __shared__ __align__(16) uint16_t lds_idx_raw[C];
    const KeyPlain<KW> lds_key{lds_key_raw};
    const IdxPlain<KW> lds_idx{lds_idx_raw};
    __shared__ uint32_t cnt[LeafShape<KW>::CNT_WORDS];
    __shared__ uint32_t tmp[NW];
    __shared__ uint64_t tmp64[NW];

    // Wide leaves (one block per CU either way) also park their row ids in
    // LDS, loaded together with the keys: one memory latency instead of two.
    constexpr bool PARK = sizeof(KW) == 8;
    __shared__ int32_t lds_rid_park[PARK ? C : 1];

    const LeafDesc L = leaves[blockIdx.x];
    if (L.rn == 0) return;
    const K* __restrict__ src_k = (const K*)bufs.key[L.buf][0] + L.kr0;
    const int32_t* __restrict__ src_r = bufs.rid[L.buf][0] + L.r0;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;
    KW key[KI];
    int32_t prid[PARK ? KI : 1];
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        const K v = ld_clamp(src_k, q, L.rn);
        if (PARK) prid[PARK ? r : 0] = ld_clamp(src_r, threadIdx.x + r * NT, L.rn);
        key[r] = q < L.rn ? (KW)(ord_of(v) - L.base) : (KW)~(KW)0;
    }
    if (PARK) {
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = threadIdx.x + r * NT;
            if (q < L.rn) lds_rid_park[q] = prid[PARK ? r : 0];
        }
    }
    uint16_t idx[KI];
#pragma unroll
    for (int r = 0; r < KI; r++) idx[r] = (uint16_t)((w * KI + r) * 64 + l);
    if (L.bits > 0 &&
        block_bin_sort<KW, NT, KI, LeafShape<KW>::NBB>(key, (int)L.bits, L.rn, lds_key, lds_idx, cnt, tmp)) {
        // sorted in one counting pass
    } else if (sizeof(KW) == 8 && L.bits > 32) {
        // Wide keys: sort by the top 32 bits of the relative key only (4 digit
        // passes instead of up to 8). The order is final unless two rows share
        // those 32 bits; short runs of such ties are then put in order by one
        // thread each (insertion sort on the full key, which keeps equal keys in
        // input order); many ties fall back to the full sort.
        const int H = (int)L.bits - 32;
        block_lsd_sort<KW, NT, KI>(key, idx, 32, lds_key, lds_idx, cnt, tmp, H);
        uint32_t ties = 0;
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = threadIdx.x * KI + r;
            if (q > 0 && q < L.rn && (lds_key[q] >> H) == (lds_key[q - 1] >> H)) ties++;
        }
        ties = (uint32_t)block_sum64<NT>((uint64_t)ties, tmp64);
        if (ties > 0 && ties <= 256) {
#pragma unroll
            for (int r = 0; r < KI; r++) {
                const uint32_t q = threadIdx.x * KI + r;
                const bool head = q + 1 < L.rn && (lds_key[q] >> H) == (lds_key[q + 1] >> H) &&
                                  (q == 0 || (lds_key[q] >> H) != (lds_key[q - 1] >> H));
                if (!head) continue;
                uint32_t e = q + 1;
                while (e < L.rn && (lds_key[e] >> H) == (lds_key[q] >> H)) e++;
                for (uint32_t i = q + 1; i < e; i++) {  // stable insertion sort of [q, e)
                    const KW kv = lds_key[i];
                    const uint16_t iv = lds_idx[i];
                    uint32_t j = i;
                    while (j > q && lds_key[j - 1] > kv) {
                        lds_key[j] = lds_key[j - 1];
                        lds_idx[j] = lds_idx[j - 1];
                        j--;
                    }
                    lds_key[j] = kv;
                    lds_idx[j] = iv;
                }
            }
            lds_barrier();
        } else if (ties > 256) {
#pragma unroll
            for (int r = 0; r < KI; r++) {
                const uint32_t q = (w * KI + r) * 64 + l;
                const K v = ld_clamp(src_k, q, L.rn);
        key[r] = q < L.rn ? (KW)(ord_of(v) - L.base) : (KW)~(KW)0;
                idx[r] = (uint16_t)q;
            }
            block_lsd_sort<KW, NT, KI>(key, idx, (int)L.bits, lds_key, lds_idx, cnt, tmp);
        }
    } else {
        block_lsd_sort<KW, NT, KI>(key, idx, (int)L.bits, lds_key, lds_idx, cnt, tmp);
    }
    // Keys go out first. The bucket may be sorted in place (its rows already
    // sit in the output columns), so its row ids are all read (coalesced, into
    // the now free key array) before any of them is overwritten.
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        if (q < L.rn) out_k[L.out + q] = key_of<K>(L.base + (uint64_t)lds_key[q]);
    }
    int32_t* lds_rid = PARK ? lds_rid_park : (int32_t*)lds_key_raw;
    if (!PARK) {
        lds_barrier();
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = threadIdx.x + r * NT;
            const int32_t v = ld_clamp(src_r, q, L.rn);
            if (q < L.rn) lds_rid[q] = v;
        }
        lds_barrier();
    }
#pragma unroll
    for (int r = 0; r < KI; r++) {
        const uint32_t q = (w * KI + r) * 64 + l;
        if (q < L.rn) out_r[L.out + q] = lds_rid[lds_idx[q]];
    }
}

hipError_t launch_leaf_sort(int key_bytes, bool wide, const LeafDesc* leaves, uint32_t n,
                            BufSet bufs, void* out_k, int32_t* out_r, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 grid(n), block(wide ? LeafShape<uint64_t>::NT : LeafShape<uint32_t>::NT);
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
//
// Count mode adds the block's pair count to *total. Materialise mode takes a
// ticket (so blocks handle buckets in key order), publishes its pair count,
// and finds its output offset by decoupled look-back over the published
// counts of the buckets before it; status[0] holds the offset carried in.
// Pairs at or beyond `capacity` are not written.
// ---------------------------------------------------------------------------
constexpr uint64_t ST_AGG = 1ull << 62, ST_INC = 2ull << 62, ST_VAL = (1ull << 62) - 1;
constexpr uint64_t LOOKBACK_SPIN_LIMIT = 1ull << 22;
constexpr uint32_t COOP_PAIRS = 16;  // R rows with more pairs are written by their whole wave

template <typename KW>
__device__ __forceinline__ uint32_t lds_upper_bound(const KW* a, uint32_t lo, uint32_t hi, KW k)
{
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (a[m] <= k) lo = m + 1; else hi = m;
    }
    return lo;
}

// A status word carries its whole message (flag and value in one 64-bit word)
// and no other data is published through it, so relaxed device-scope atomics
// suffice: release/acquire would make every block wait for its earlier
// memory operations and write back or invalidate its L2 (each XCD has its
// own) on the way.
__device__ __forceinline__ void status_store(uint64_t* p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t status_load(const uint64_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of bucket `slot - 1` (slot >= 1), computed by one whole
// wave: lane i reads status[hi - i] for a window of 64 predecessors. The window
// is summed from its newest entry down to the nearest inclusive prefix; if the
// window holds only aggregates it is summed whole and the walk moves 64 slots
// back. A window is re-read while any entry it needs is unpublished. Every
// predecessor already holds its ticket, so it is running or done and will
// publish; the spin is bounded all the same, and on expiry *err is set and 0
// returned. status[0] is always an inclusive prefix, so the walk ends.
__device__ uint64_t look_back(uint64_t* status, uint32_t slot, uint32_t* err)
{
    const uint32_t l = lane_id();
    uint64_t sum = 0, spins = 0;
    int64_t hi = (int64_t)slot - 1;
    while (true) {
        const int64_t j = hi - (int64_t)l;
        const uint64_t s = j >= 0 ? status_load(&status[j]) : 0;
        const uint64_t f = s & ~ST_VAL;
        const uint64_t inc = ballot(j >= 0 && f == ST_INC);
        const uint64_t pending = ballot(j >= 0 && f == 0);
        const int first = inc ? __ffsll((unsigned long long)inc) - 1 : 64;
        const uint64_t need = first >= 63 ? ~0ull : ((2ull << first) - 1);
        if (pending & need) {
            if (++spins > LOOKBACK_SPIN_LIMIT) {
                if (l == 0) atomicOr(err, 1u);
                return 0;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        sum += wave_sum64(((need >> l) & 1ull) && j >= 0 ? (s & ST_VAL) : 0ull);
        if (first < 64) return sum;
        hi -= 64;
    }
}

template <typename K, typename KW, bool MAT>
__global__ __launch_bounds__(LeafShape<KW>::NT)
__attribute__((amdgpu_waves_per_eu(4))) void k_leaf_join(const LeafDesc* __restrict__ leaves,
                                                            BufSet bufs, uint64_t* __restrict__ status,
                                                            uint32_t* __restrict__ ticket,
                                                            uint64_t* __restrict__ total,
                                                            uint32_t* __restrict__ err,
                                                            int32_t* __restrict__ out_r,
                                                            int32_t* __restrict__ out_s,
                                                            uint64_t capacity)
{
    constexpr int NT = LeafShape<KW>::NT, KI = LeafShape<KW>::KI, NW = LeafShape<KW>::NW, C = LEAF_CAP;
    // (padded for the count; the materialising block keeps the plain layout:
    // the padding's address arithmetic costs it registers it does not have)
    using KA = typename std::conditional<MAT, KeyPlain<KW>, KeyLds<KW>>::type;
    using IA = typename std::conditional<MAT, IdxPlain<KW>, IdxLds<KW>>::type;
    __shared__ KW lds_key_raw[KA::size(C)];
    __shared__ __align__(16) uint16_t lds_idx_raw[IA::size(C)];
    const KA lds_key{lds_key_raw};
    const IA lds_idx{lds_idx_raw};
    __shared__ uint32_t cnt[NW * LSTRIDE];
    __shared__ uint32_t tmp[NW];
    __shared__ uint64_t tmp64[NW];
    __shared__ uint32_t s_leaf;
    __shared__ uint64_t s_base;
    __shared__ uint32_t s_unordered;

    if (threadIdx.x == 0) s_unordered = 0;
    uint32_t li = blockIdx.x;
    if (MAT) {
        if (threadIdx.x == 0) s_leaf = atomicAdd(ticket, 1u);
        lds_barrier();
        li = s_leaf;
    }
    const LeafDesc L = leaves[li];
    const uint32_t rn = L.rn, n = L.rn + L.sn;
    const K* __restrict__ rk = (const K*)bufs.key[L.buf][0] + L.kr0;
    const K* __restrict__ sk = (const K*)bufs.key[L.buf][1] + L.ks0;
    const uint32_t w = threadIdx.x / 64, l = threadIdx.x & 63;

    KW key[KI];
    uint16_t idx[KI];
    auto load_items = [&]() {
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = (w * KI + r) * 64 + l;
            key[r] = (KW)~(KW)0;
            idx[r] = (uint16_t)q;
        }
        if (n > 0) {
#pragma unroll
            for (int r = 0; r < KI; r++) {
                const uint32_t q = (w * KI + r) * 64 + l;
                const uint32_t qc = q < n ? q : n - 1;  // every lane loads a real row
                const K v = qc < rn ? rk[qc] : sk[qc - rn];
                if (q < n) key[r] = (KW)(ord_of(v) - L.base);
            }
        }
    };
    // (LSD rather than block_bin_sort: a key here usually has several rows, one
    // of R and its S matches, which makes the bins too full for the exact
    // in-bin ranking to pay.) Ranked by atomics, then checked; sorted again
    // with ballot ranking if the order is not exact.
    load_items();
    block_lsd_sort<KW, NT, KI, true>(key, idx, (int)L.bits, lds_key, lds_idx, cnt, tmp);
    if (!block_check_order<KW, NT, KI>(lds_key, lds_idx, n, &s_unordered) || (L.flags & LEAF_FORCE_REORDER)) {
        load_items();
        block_lsd_sort<KW, NT, KI, false>(key, idx, (int)L.bits, lds_key, lds_idx, cnt, tmp);
    }

    // Run analysis on blocked positions p = tid*KI + i. A run is a maximal
    // stretch of equal keys: [rs, s0) holds its a R items, [s0, re) its b S
    // items. rs comes from a block-wide max-scan of run starts; s0 and re are
    // written, indexed by rs, by the run's last R item (or its first item when
    // the run has no R item) and by its last item.
    const uint32_t p0 = threadIdx.x * KI;
    KW kk[KI];
    uint32_t id[KI];
    lds_idx.blk_all(threadIdx.x, id);
#pragma unroll
    for (int i = 0; i < KI; i++) kk[i] = lds_key.blk(threadIdx.x, i);
    const KW kprev = p0 ? lds_key.blk(threadIdx.x - 1, KI - 1) : (KW)0;
    const KW knext = p0 + KI < C ? lds_key.blk(threadIdx.x + 1, 0) : (KW)0;
    const uint32_t inext = p0 + KI < C ? lds_idx.blk(threadIdx.x + 1, 0) : 0xffffu;
    uint32_t rs[KI];
    uint32_t run_start = 0;
#pragma unroll
    for (int i = 0; i < KI; i++) {
        const uint32_t p = p0 + i;
        const bool start = p == 0 || p >= n || kk[i] != (i ? kk[i - 1] : kprev);
        run_start = start ? p : run_start;
        rs[i] = run_start;
    }
    {
        const uint32_t carry = block_excl_max<NT>(run_start, tmp);  // barriers: keys all read
#pragma unroll
        for (int i = 0; i < KI; i++) rs[i] = max(rs[i], carry);
    }
    uint16_t* run_s0 = (uint16_t*)lds_key_raw;   // the key array is free from here on
    uint16_t* run_end = run_s0 + C;
#pragma unroll
    for (int i = 0; i < KI; i++) {
        const uint32_t p = p0 + i;
        if (p >= n) continue;
        const bool last = p == n - 1 || (i + 1 < KI ? kk[i + 1] : knext) != kk[i];
        const uint32_t idn = i + 1 < KI ? id[i + 1] : inext;
        const bool isr = id[i] < rn;
        if (last) run_end[rs[i]] = (uint16_t)(p + 1);
        if (isr && (last || idn >= rn)) run_s0[rs[i]] = (uint16_t)(p + 1);   // last R item
        if (!isr && p == rs[i]) run_s0[rs[i]] = (uint16_t)p;                  // run without R items
    }
    lds_barrier();
    // per item, packed: [is R:1][a:14][b:14], a = R items and b = S items of its
    // run (0 for padding); kv = position of the item inside the run's S part
    uint32_t abv[KI], kv[KI];
    uint32_t local = 0;
#pragma unroll
    for (int i = 0; i < KI; i++) {
        abv[i] = 0;
        kv[i] = 0;
        if (p0 + i < n) {
            const uint32_t s0 = run_s0[rs[i]], re = run_end[rs[i]];
            const uint32_t a = s0 - rs[i], b = re - s0;
            const bool isr = id[i] < rn;
            abv[i] = (isr ? 0x80000000u : 0u) | (a << 14) | b;
            kv[i] = p0 + i - s0;
            if (isr) local += b;  // an R item owns b pairs
        }
    }
    if (!MAT) {
        const uint64_t c = block_sum64<NT>((uint64_t)local, tmp64);
        if (threadIdx.x == 0 && c) atomicAdd((unsigned long long*)total, (unsigned long long)c);
        return;
    }
    uint32_t ltot;
    uint32_t ex = block_excl_scan<NT>(local, tmp, &ltot);  // barriers: run tables all read
    if (threadIdx.x == 0) status_store(&status[li + 1], ST_AGG | (uint64_t)ltot);
    // Row ids: one coalesced load of the block's rows (R then S) into the free
    // key array, then every item picks its own from LDS.
    int32_t* lds_w = (int32_t*)lds_key_raw;
    {
        const int32_t* __restrict__ rr = bufs.rid[L.buf][0] + L.r0;
        const int32_t* __restrict__ sr = bufs.rid[L.buf][1] + L.s0;
#pragma unroll
        for (int r = 0; r < KI; r++) {
            const uint32_t q = threadIdx.x + r * NT;
            const uint32_t qc = q < n ? q : n - 1;
            const int32_t v = qc < rn ? rr[qc] : sr[qc - rn];
            if (q < n) lds_w[q] = v;
        }
    }
    if (threadIdx.x < 64) {
        const uint64_t excl = look_back(status, li + 1, err);
        if (threadIdx.x == 0) {
            status_store(&status[li + 1], ST_INC | (excl + ltot));
            s_base = excl + L.out;
        }
    }
    lds_barrier();
    const uint64_t base = s_base;
    // Pair slots: R item j of a run owns E_rs + j*b .. + b (it writes out_r),
    // S item k of a run appears at E_rs + i*b + k for its run's a R items (it
    // writes out_s). Per item: first slot, and packed [side:1][slots:14][stride:14].
    uint32_t firstv[KI], packv[KI];
    uint32_t maxslots = 0;
    {
        uint32_t e = ex;
#pragma unroll
        for (int i = 0; i < KI; i++) {
            const uint32_t ab = abv[i];
            const bool isr = (ab >> 31) != 0;
            const uint32_t a = (ab >> 14) & 0x3fffu, b = ab & 0x3fffu;
            const uint32_t slots = isr ? b : (b ? a : 0u);
            const uint32_t stride = isr ? 1u : b;
            packv[i] = (isr ? 0x80000000u : 0u) | (slots << 14) | stride;
            firstv[i] = isr ? e : e - a * b + kv[i];
            maxslots = slots > maxslots ? slots : maxslots;
            if (isr) e += b;
        }
    }
    maxslots = block_max<NT>(maxslots, tmp);
    int32_t rid[KI];
#pragma unroll
    for (int i = 0; i < KI; i++) rid[i] = p0 + i < n ? lds_w[id[i]] : 0;
    lds_barrier();  // the key array becomes the pair staging buffer
    constexpr uint32_t SC = C * sizeof(KW) / 4;  // int32 slots of the key array
    if (ltot <= 4 * SC && maxslots <= 64) {
        // Staged, one output column at a time: that column's items scatter
        // their slots of the chunk into LDS, then the chunk leaves as one
        // coalesced run. An R item's slots are consecutive, so it visits only
        // those inside the chunk.
        int32_t* st = lds_w;
        for (int side = 0; side < 2; side++) {
            int32_t* __restrict__ dst = side ? out_s : out_r;
            for (uint32_t c0 = 0; c0 < ltot; c0 += SC) {
                const uint32_t c1 = c0 + SC;
#pragma unroll
                for (int i = 0; i < KI; i++) {
                    const uint32_t pk = packv[i];
                    const uint32_t sl = (pk >> 14) & 0x3fffu, stride = pk & 0x3fffu;
                    const uint32_t f = firstv[i];
                    if (side == 0 && (pk >> 31)) {
                        const uint32_t j0 = f < c0 ? c0 - f : 0u;
                        const uint32_t j1 = f + sl < c1 ? sl : (c1 > f ? c1 - f : 0u);
                        for (uint32_t j = j0; j < j1; j++) st[f + j - c0] = rid[i];
                    } else if (side == 1 && !(pk >> 31)) {
                        for (uint32_t j = 0; j < sl; j++) {
                            const uint32_t t = f + j * stride;
                            if (t >= c0 && t < c1) st[t - c0] = rid[i];
                        }
                    }
                }
                lds_barrier();
                const uint32_t cn = ltot - c0 < SC ? ltot - c0 : SC;
                for (uint32_t t = threadIdx.x; t < cn; t += NT) {
                    const uint64_t o = base + c0 + t;
                    if (o < capacity) dst[o] = st[t];
                }
                lds_barrier();
            }
        }
        return;
    }
    // Very large outputs (hot keys inside the block): items write their own
    // slots; items with many slots are written by their wave.
#pragma unroll
    for (int i = 0; i < KI; i++) {
        const uint32_t pk = packv[i];
        const uint32_t slots = (pk >> 14) & 0x3fffu, stride = pk & 0x3fffu, first = firstv[i];
        int32_t* __restrict__ dst = (pk >> 31) ? out_r : out_s;
        if (slots && slots <= COOP_PAIRS) {
            for (uint32_t j = 0; j < slots; j++) {
                const uint64_t t = base + first + (uint64_t)j * stride;
                if (t < capacity) dst[t] = rid[i];
            }
        }
        uint64_t m = ballot(slots > COOP_PAIRS);
        while (m) {
            const int src = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            const uint32_t cpk = __shfl(pk, src, 64);
            const uint32_t cs = (cpk >> 14) & 0x3fffu, cst = cpk & 0x3fffu;
            const uint32_t cf = __shfl(first, src, 64);
            const int32_t cr = __shfl(rid[i], src, 64);
            int32_t* __restrict__ cdst = (cpk >> 31) ? out_r : out_s;
            for (uint32_t j = l; j < cs; j += 64) {
                const uint64_t t = base + cf + (uint64_t)j * cst;
                if (t < capacity) cdst[t] = cr;
            }
        }
    }
}

hipError_t launch_leaf_join(int key_bytes, bool wide, bool materialize, const LeafDesc* leaves,
                            uint32_t n, BufSet bufs, uint64_t* status, uint32_t* ticket,
                            uint64_t* total, uint32_t* err, int32_t* out_r, int32_t* out_s,
                            uint64_t capacity, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const dim3 grid(n), block(wide ? LeafShape<uint64_t>::NT : LeafShape<uint32_t>::NT);
#define TJ_LJ(K, KW, M)                                                                              \
    hipLaunchKernelGGL((k_leaf_join<K, KW, M>), grid, block, 0, st, leaves, bufs, status, ticket,    \
                       total, err, out_r, out_s, capacity)
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
// each block takes a fixed stretch of it. A unit's output offset is the
// inclusive pair prefix of the per-bucket joins before it (status, after the
// materialising leaf launch) plus the pairs of earlier single-key units.
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
                                                         const uint64_t* __restrict__ status,
                                                         int32_t* __restrict__ out_r,
                                                         int32_t* __restrict__ out_s,
                                                         uint64_t capacity)
{
    const uint64_t t0 = blockIdx.x * CROSS_PER_BLOCK;
    uint64_t t1 = t0 + CROSS_PER_BLOCK;
    if (t1 > total) t1 = total;
    const size_t stride = sizeof(CrossDesc) / 8;
    const uint64_t* pfx = &units[0].pfx;
    uint64_t t = t0 + threadIdx.x;
    if (t >= t1) return;
    uint32_t u = find_unit(pfx, stride, n, t);
    CrossDesc U;
    uint64_t base = 0, end = 0, i = 0, j = 0;
    uint32_t qi = 0, qj = 0;  // a step of CROSS_THREADS pairs moves (i, j) by (qi, qj), then carries
    // pair loc = t - pfx of the unit is (R row i, S row j) with loc = i*b + j;
    // only a thread's first pair of a unit divides, later pairs step
    auto enter = [&]() {
        U = units[u];
        base = U.out + (status[U.leaf_before] & ST_VAL);
        end = U.pfx + U.a * U.b;
        const uint64_t loc = t - U.pfx;
        i = (uint64_t)((double)loc / (double)U.b);
        while (i * U.b > loc) i--;
        while ((i + 1) * U.b <= loc) i++;
        j = loc - i * U.b;
        qi = U.b > CROSS_THREADS ? 0u : (uint32_t)(CROSS_THREADS / U.b);
        qj = (uint32_t)(CROSS_THREADS - (uint64_t)qi * U.b);
    };
    auto step = [&](uint64_t& si, uint64_t& sj) {
        si += qi;
        sj += qj;
        if (sj >= U.b) {
            sj -= U.b;
            si++;
        }
    };
    constexpr int UNR = 4;  // pairs per thread whose row-id loads are issued together
    enter();
    while (t < t1) {
        if (t >= end) {
            do ++u; while (t >= units[u].pfx + units[u].a * units[u].b);
            enter();
        }
        const int32_t* __restrict__ rr = bufs.rid[U.buf][0] + U.r0;
        const int32_t* __restrict__ sr = bufs.rid[U.buf][1] + U.s0;
        const uint64_t last = t + (UNR - 1) * (uint64_t)CROSS_THREADS;
        if (last < end && last < t1) {
            uint64_t ii[UNR], jj[UNR];
            ii[0] = i;
            jj[0] = j;
#pragma unroll
            for (int k = 1; k < UNR; k++) {
                ii[k] = ii[k - 1];
                jj[k] = jj[k - 1];
                step(ii[k], jj[k]);
            }
            int32_t vr[UNR], vs[UNR];
#pragma unroll
            for (int k = 0; k < UNR; k++) {
                vr[k] = rr[ii[k]];
                vs[k] = sr[jj[k]];
            }
#pragma unroll
            for (int k = 0; k < UNR; k++) {
                const uint64_t o = base + (t + k * (uint64_t)CROSS_THREADS - U.pfx);
                if (o < capacity) {
                    out_r[o] = vr[k];
                    out_s[o] = vs[k];
                }
            }
            i = ii[UNR - 1];
            j = jj[UNR - 1];
            step(i, j);
            t += UNR * (uint64_t)CROSS_THREADS;
        } else {
            const uint64_t o = base + (t - U.pfx);
            if (o < capacity) {
                out_r[o] = rr[i];
                out_s[o] = sr[j];
            }
            step(i, j);
            t += CROSS_THREADS;
        }
    }
}

hipError_t launch_cross(const CrossDesc* units, uint32_t n, uint64_t total, BufSet bufs,
                        const uint64_t* status, int32_t* out_r, int32_t* out_s, uint64_t capacity,
                        hipStream_t st)
{
    if (n == 0 || total == 0) return hipSuccess;
    const uint64_t blocks = (total + CROSS_PER_BLOCK - 1) / CROSS_PER_BLOCK;
    hipLaunchKernelGGL(k_cross, dim3((uint32_t)blocks), dim3(CROSS_THREADS), 0, st, units, n, total,
                       bufs, status, out_r, out_s, capacity);
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

// tj_fuse.hip - gather and scatter kernels of the serving loop's fused calls.
//
// Several small requests of one kind run as one composite-key call whose
// leading key column is the request's index in the batch: request i's rows
// then stay together and in their own order (sort), and its pairs form one
// contiguous stretch in its own canonical order (join), because the index
// column is compared first. These kernels build the combined columns and
// hand every request its part of the result.
#include "tj_internal.h"

namespace tj {

namespace {

constexpr int FUSE_THREADS = 256;

// Combined columns: rows [off, off + n) of one side take request i's keys, the
// index i and, as row ids, the request's own row ids or (positions != 0) the
// rows' positions in the combined relation.
template <typename K>
__global__ __launch_bounds__(FUSE_THREADS) void k_fuse_gather(const FuseDesc* __restrict__ desc, int side,
                                                              int positions, int32_t* __restrict__ item,
                                                              K* __restrict__ keys, int32_t* __restrict__ rids)
{
    const FuseDesc d = desc[blockIdx.y];
    const uint64_t n = side ? d.n_s : d.n_r, off = side ? d.off_s : d.off_r;
    const K* __restrict__ src = (const K*)(side ? d.s_keys : d.r_keys);
    const int32_t* __restrict__ srid = side ? d.s_rids : d.r_rids;
    for (uint64_t i = blockIdx.x * (uint64_t)FUSE_THREADS + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * FUSE_THREADS) {
        item[off + i] = (int32_t)blockIdx.y;
        keys[off + i] = src[i];
        rids[off + i] = positions ? (int32_t)(off + i) : srid[i];
    }
}

// Sort results: request i's rows sit at [d.off_r, d.off_r + d.n_r) of the
// sorted combined columns (the request index is the leading key).
template <typename K>
__global__ __launch_bounds__(FUSE_THREADS) void k_fuse_scatter_sort(const FuseDesc* __restrict__ desc,
                                                                    const K* __restrict__ keys,
                                                                    const int32_t* __restrict__ rids)
{
    const FuseDesc d = desc[blockIdx.y];
    K* __restrict__ ok = (K*)d.out0;
    for (uint64_t i = blockIdx.x * (uint64_t)FUSE_THREADS + threadIdx.x; i < d.n_r;
         i += (uint64_t)gridDim.x * FUSE_THREADS) {
        ok[i] = keys[d.off_r + i];
        d.out1[i] = rids[d.off_r + i];
    }
}

// Join boundaries: bounds[i] = first pair whose R row belongs to a request
// >= i (pairs are ordered by request index first); bounds[nreq] = count.
__global__ void k_fuse_bounds(const int32_t* __restrict__ pr, const int32_t* __restrict__ item_r,
                              uint64_t count, uint32_t nreq, uint64_t* __restrict__ bounds)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nreq) return;
    uint64_t lo = 0, hi = count;
    while (lo < hi) {
        const uint64_t m = lo + (hi - lo) / 2;
        if ((uint32_t)item_r[pr[m]] < i) lo = m + 1; else hi = m;
    }
    bounds[i] = i == nreq ? count : lo;
}

// Join results: pair t of request i (bounds[i] <= t < bounds[i+1]) is written
// at t - bounds[i] as the request's own row ids, when all the request's pairs
// fit its capacity (otherwise the request writes nothing).
__global__ __launch_bounds__(FUSE_THREADS) void k_fuse_scatter_pairs(const FuseDesc* __restrict__ desc,
                                                                     uint32_t nreq,
                                                                     const uint64_t* __restrict__ bounds,
                                                                     const int32_t* __restrict__ pr,
                                                                     const int32_t* __restrict__ ps,
                                                                     uint64_t count)
{
    for (uint64_t t = blockIdx.x * (uint64_t)FUSE_THREADS + threadIdx.x; t < count;
         t += (uint64_t)gridDim.x * FUSE_THREADS) {
        uint32_t lo = 0, hi = nreq;  // last request with bounds <= t
        while (hi - lo > 1) {
            const uint32_t m = (lo + hi) / 2;
            if (bounds[m] <= t) lo = m; else hi = m;
        }
        const FuseDesc d = desc[lo];
        if (bounds[lo + 1] - bounds[lo] > d.capacity) continue;
        const uint64_t j = t - bounds[lo];
        ((int32_t*)d.out0)[j] = d.r_rids[(uint64_t)pr[t] - d.off_r];
        d.out1[j] = d.s_rids[(uint64_t)ps[t] - d.off_s];
    }
}

dim3 grid_for(uint64_t max_rows, uint32_t nreq)
{
    uint64_t bx = (max_rows + FUSE_THREADS - 1) / FUSE_THREADS;
    if (bx < 1) bx = 1;
    if (bx > 1024) bx = 1024;
    return dim3((uint32_t)bx, nreq);
}

}  // namespace

hipError_t launch_fuse_gather(int key_bytes, const FuseDesc* desc, uint32_t nreq, uint64_t max_rows, int side,
                              int positions, int32_t* item, void* keys, int32_t* rids, hipStream_t st)
{
    if (nreq == 0) return hipSuccess;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_fuse_gather<int32_t>, grid_for(max_rows, nreq), dim3(FUSE_THREADS), 0, st, desc, side,
                           positions, item, (int32_t*)keys, rids);
    else
        hipLaunchKernelGGL(k_fuse_gather<int64_t>, grid_for(max_rows, nreq), dim3(FUSE_THREADS), 0, st, desc, side,
                           positions, item, (int64_t*)keys, rids);
    return hipGetLastError();
}

hipError_t launch_fuse_scatter_sort(int key_bytes, const FuseDesc* desc, uint32_t nreq, uint64_t max_rows,
                                    const void* keys, const int32_t* rids, hipStream_t st)
{
    if (nreq == 0) return hipSuccess;
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_fuse_scatter_sort<int32_t>, grid_for(max_rows, nreq), dim3(FUSE_THREADS), 0, st, desc,
                           (const int32_t*)keys, rids);
    else
        hipLaunchKernelGGL(k_fuse_scatter_sort<int64_t>, grid_for(max_rows, nreq), dim3(FUSE_THREADS), 0, st, desc,
                           (const int64_t*)keys, rids);
    return hipGetLastError();
}

hipError_t launch_fuse_bounds(const int32_t* pr, const int32_t* item_r, uint64_t count, uint32_t nreq,
                              uint64_t* bounds, hipStream_t st)
{
    hipLaunchKernelGGL(k_fuse_bounds, dim3((nreq + 1 + 63) / 64), dim3(64), 0, st, pr, item_r, count, nreq, bounds);
    return hipGetLastError();
}

hipError_t launch_fuse_scatter_pairs(const FuseDesc* desc, uint32_t nreq, const uint64_t* bounds, const int32_t* pr,
                                     const int32_t* ps, uint64_t count, hipStream_t st)
{
    if (count == 0 || nreq == 0) return hipSuccess;
    uint64_t blocks = (count + FUSE_THREADS - 1) / FUSE_THREADS;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fuse_scatter_pairs, dim3((uint32_t)blocks), dim3(FUSE_THREADS), 0, st, desc, nreq, bounds,
                       pr, ps, count);
    return hipGetLastError();
}

}  // namespace tj

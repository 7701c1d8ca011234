// tj_bandwidth.hip - a plain streaming copy: the bandwidth a read-once,
// write-once kernel reaches on this device, the "achievable" line the other
// kernels are compared with.
#include "tj_internal.h"

namespace tj {

namespace {

constexpr int COPY_THREADS = 256;
constexpr int COPY_UNROLL = 4;  // 16-byte loads in flight per thread

__global__ __launch_bounds__(COPY_THREADS) void k_stream_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                              uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * COPY_THREADS;
    uint64_t i = blockIdx.x * (uint64_t)COPY_THREADS + threadIdx.x;
    for (; i + (COPY_UNROLL - 1) * stride < n; i += COPY_UNROLL * stride) {
        uint4 v[COPY_UNROLL];
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; u++) v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; u++) dst[i + u * stride] = v[u];
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t st)
{
    const uint64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    uint64_t blocks = (uint64_t)cus * 8;  // 8 blocks of 4 waves per CU
    const uint64_t need = (n + COPY_THREADS - 1) / COPY_THREADS;
    if (blocks > need) blocks = need;
    hipLaunchKernelGGL(k_stream_copy, dim3((uint32_t)blocks), dim3(COPY_THREADS), 0, st, (const uint4*)src, (uint4*)dst,
                       n);
    return hipGetLastError();
}

}  // namespace tj

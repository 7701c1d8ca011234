// tj_rmi.hip - training and evaluation kernels of the learned CDF partitioner
// (the model is defined in tj.h, tj_rmi_t). Training runs on the sorted sample:
//   k_rmi_sample  gathers the sample rows of a relation (positions floor(i n / m));
//   (the plain sort path sorts the sample)
//   k_rmi_root    equal-depth knots of the sorted sample and their f32 inverses;
//   k_rmi_route   routes every sample point through the root and records where
//                 each leaf's run of points starts (the sample is sorted and the
//                 root is monotone, so a leaf's points are contiguous);
//   k_rmi_fit     one block per leaf: least-squares line in fp64, stored as f32;
//   k_rmi_fill    bucket interval of every leaf, empty leaves included.
// None of it is on the bandwidth-bound path: the sample is 1% of the rows.
#include <hip/hip_runtime.h>
#include <cstdint>

#include "tj_internal.h"
#include "tj_rmi.h"

namespace tj {
namespace {

__device__ __forceinline__ uint64_t rmi_ord(int32_t k) { return (uint64_t)((uint32_t)k ^ 0x80000000u); }
__device__ __forceinline__ uint64_t rmi_ord(int64_t k) { return (uint64_t)k ^ 0x8000000000000000ull; }

template <typename K>
__global__ __launch_bounds__(256) void k_rmi_sample(const K* __restrict__ keys, uint64_t n, uint32_t m,
                                                    K* __restrict__ out, int32_t* __restrict__ rids,
                                                    uint32_t off)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < m; i += gridDim.x * 256) {
        const uint64_t pos = (uint64_t)i * n / m;  // < n; i * n < 2^62
        out[off + i] = keys[pos];
        rids[off + i] = (int32_t)(off + i);
    }
}

template <typename K>
__global__ __launch_bounds__(256) void k_rmi_root(const K* __restrict__ s, uint32_t M, uint32_t F,
                                                  tj_rmi_t* __restrict__ model)
{
    for (uint32_t i = threadIdx.x; i <= TJ_RMI_SEGMENTS; i += 256) {
        const uint64_t at = (uint64_t)i * (M - 1) / TJ_RMI_SEGMENTS;
        const uint64_t k = rmi_ord(s[at]);
        model->knot[i] = k;
        if (i < TJ_RMI_SEGMENTS) {
            const uint64_t k1 = rmi_ord(s[(uint64_t)(i + 1) * (M - 1) / TJ_RMI_SEGMENTS]);
            model->knot_inv[i] = k1 > k ? (float)(1.0 / (double)(k1 - k)) : 0.0f;
        }
    }
    if (threadIdx.x == 0) {
        model->buckets = F;
        model->sample_rows = M;
    }
}

// start[l] = first sample index whose leaf is >= l, for l in [0, LEAVES]
template <typename K>
__global__ __launch_bounds__(256) void k_rmi_route(const K* __restrict__ s, uint32_t M,
                                                   const tj_rmi_t* __restrict__ model,
                                                   uint32_t* __restrict__ start)
{
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i <= M; i += gridDim.x * 256) {
        const int32_t cur = i < M ? (int32_t)rmi_leaf(*model, rmi_ord(s[i])) : TJ_RMI_LEAVES;
        const int32_t prev = i ? (int32_t)rmi_leaf(*model, rmi_ord(s[i - 1])) : -1;
        for (int32_t l = prev + 1; l <= cur; l++) start[l] = i;
    }
}

constexpr int FIT_NT = 256;

__device__ __forceinline__ void block_sum2(double& a, double& b, double* tmp)
{
    tmp[threadIdx.x] = a;
    tmp[FIT_NT + threadIdx.x] = b;
    __syncthreads();
    for (int h = FIT_NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            tmp[threadIdx.x] += tmp[threadIdx.x + h];
            tmp[FIT_NT + threadIdx.x] += tmp[FIT_NT + threadIdx.x + h];
        }
        __syncthreads();
    }
    a = tmp[0];
    b = tmp[FIT_NT];
    __syncthreads();
}

// one block per leaf: least-squares line through (s_i - base, F i / M)
template <typename K>
__global__ __launch_bounds__(FIT_NT) void k_rmi_fit(const K* __restrict__ s, uint32_t M, uint32_t F,
                                                    const uint32_t* __restrict__ start,
                                                    tj_rmi_t* __restrict__ model)
{
    __shared__ double tmp[2 * FIT_NT];
    const uint32_t l = blockIdx.x;
    const uint32_t a = start[l], b = start[l + 1];
    if (b <= a) {
        if (threadIdx.x == 0) {
            model->leaf_base[l] = 0;
            model->leaf_a[l] = 0.0f;
            model->leaf_b[l] = 0.0f;
        }
        return;
    }
    const uint64_t base = rmi_ord(s[a]);
    const double fm = (double)F, mm = (double)M;
    double sd = 0.0, sy = 0.0;
    for (uint32_t i = a + threadIdx.x; i < b; i += FIT_NT) {
        sd += (double)(rmi_ord(s[i]) - base);
        sy += fm * (double)i / mm;
    }
    block_sum2(sd, sy, tmp);
    const double cnt = (double)(b - a);
    const double dm = sd / cnt, ym = sy / cnt;
    double sdd = 0.0, sdy = 0.0;
    for (uint32_t i = a + threadIdx.x; i < b; i += FIT_NT) {
        const double dd = (double)(rmi_ord(s[i]) - base) - dm;
        const double dy = fm * (double)i / mm - ym;
        sdd += dd * dd;
        sdy += dd * dy;
    }
    block_sum2(sdd, sdy, tmp);
    if (threadIdx.x == 0) {
        double slope = sdd > 0.0 ? sdy / sdd : 0.0;
        if (!(slope > 0.0)) slope = 0.0;
        model->leaf_base[l] = base;
        model->leaf_b[l] = (float)slope;
        model->leaf_a[l] = (float)(ym - slope * dm);
    }
}

// bucket interval of each leaf: [F a / M, F (b - 1) / M] for its points [a, b);
// a leaf without points takes the next non-empty leaf's lower end (F - 1 if none)
__global__ __launch_bounds__(TJ_RMI_LEAVES) void k_rmi_fill(uint32_t M, uint32_t F,
                                                            const uint32_t* __restrict__ start,
                                                            tj_rmi_t* __restrict__ model)
{
    __shared__ uint32_t st[TJ_RMI_LEAVES + 1];
    for (uint32_t i = threadIdx.x; i <= TJ_RMI_LEAVES; i += TJ_RMI_LEAVES) st[i] = start[i];
    __syncthreads();
    const uint32_t l = threadIdx.x;
    uint32_t lo, hi;
    if (st[l + 1] > st[l]) {
        lo = (uint32_t)((uint64_t)F * st[l] / M);
        hi = (uint32_t)((uint64_t)F * (st[l + 1] - 1) / M);
    } else {
        uint32_t k = l + 1;
        while (k < TJ_RMI_LEAVES && st[k + 1] <= st[k]) k++;
        lo = hi = k < TJ_RMI_LEAVES ? (uint32_t)((uint64_t)F * st[k] / M) : F - 1;
    }
    model->leaf_lo[l] = (uint16_t)lo;
    model->leaf_hi[l] = (uint16_t)hi;
}

template <typename K>
__global__ __launch_bounds__(256) void k_rmi_eval(const K* __restrict__ keys, uint64_t n,
                                                  const tj_rmi_t* __restrict__ model,
                                                  uint16_t* __restrict__ out)
{
    __shared__ tj_rmi_t lm;
    rmi_to_lds<256>(&lm, model);
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        out[i] = (uint16_t)rmi_bucket(lm, rmi_ord(keys[i]));
}

inline uint32_t grid_for(uint64_t n, uint32_t cap)
{
    const uint64_t g = (n + 255) / 256;
    return (uint32_t)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_rmi_sample(int key_bytes, const void* keys, uint64_t n, uint32_t m, void* out,
                             int32_t* rids, uint32_t off, hipStream_t st)
{
    if (m == 0) return hipSuccess;
    const uint32_t g = grid_for(m, 4096);
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_rmi_sample<int32_t>, dim3(g), dim3(256), 0, st, (const int32_t*)keys, n, m,
                           (int32_t*)out, rids, off);
    else
        hipLaunchKernelGGL(k_rmi_sample<int64_t>, dim3(g), dim3(256), 0, st, (const int64_t*)keys, n, m,
                           (int64_t*)out, rids, off);
    return hipGetLastError();
}

hipError_t launch_rmi_fit(int key_bytes, const void* sorted, uint32_t M, uint32_t F, uint32_t* start,
                          tj_rmi_t* model, hipStream_t st)
{
    if (M == 0 || F == 0 || F > (uint32_t)NB) return hipErrorInvalidValue;
    const uint32_t g = grid_for((uint64_t)M + 1, 4096);
#define TJ_FIT(K)                                                                                    \
    hipLaunchKernelGGL(k_rmi_root<K>, dim3(1), dim3(256), 0, st, (const K*)sorted, M, F, model);     \
    hipLaunchKernelGGL(k_rmi_route<K>, dim3(g), dim3(256), 0, st, (const K*)sorted, M,               \
                       (const tj_rmi_t*)model, start);                                               \
    hipLaunchKernelGGL(k_rmi_fit<K>, dim3(TJ_RMI_LEAVES), dim3(FIT_NT), 0, st, (const K*)sorted, M, F, \
                       (const uint32_t*)start, model)
    if (key_bytes == 4) {
        TJ_FIT(int32_t);
    } else {
        TJ_FIT(int64_t);
    }
#undef TJ_FIT
    hipLaunchKernelGGL(k_rmi_fill, dim3(1), dim3(TJ_RMI_LEAVES), 0, st, M, F, (const uint32_t*)start, model);
    return hipGetLastError();
}

hipError_t launch_rmi_eval(int key_bytes, const void* keys, uint64_t n, const tj_rmi_t* model,
                           uint16_t* out, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint32_t g = grid_for(n, 8192);
    if (key_bytes == 4)
        hipLaunchKernelGGL(k_rmi_eval<int32_t>, dim3(g), dim3(256), 0, st, (const int32_t*)keys, n, model, out);
    else
        hipLaunchKernelGGL(k_rmi_eval<int64_t>, dim3(g), dim3(256), 0, st, (const int64_t*)keys, n, model, out);
    return hipGetLastError();
}

}  // namespace tj

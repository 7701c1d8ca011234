// tj_static.hip - the sort for callers that cannot allocate (tj_sort_static).
//
// The call is tj_sort with a fixed workspace: a file-scope device array of
// TJ_STATIC_SCRATCH_BYTES that every GPU the library runs on holds from the
// moment the library's code object is loaded until the process ends. Host
// code never passes the array's name to a kernel or a copy (in host code it
// names a host-side stand-in); it uses the device address that
// hipGetSymbolAddress returns, fetched once per device with that device
// current and kept per device.
#include "tj_internal.h"
#include "../../include/tj.h"

#include <mutex>

namespace tj {
int sort_noalloc(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n, void* keys_out,
                 int32_t* rids_out, void* workspace, uint64_t workspace_bytes, void* stream, tj_stats_t* stats);
}

namespace {

static __device__ __align__(256) unsigned char scratch[TJ_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    std::mutex mu;         // serialises the calls on one device (each returns after its work is done)
    void* ptr = nullptr;   // device address of `scratch` on this device
};
DeviceScratch g_dev[kMaxDevices];

// Device address of the scratch array on device `dev` (current), looked up on
// the first call on that device. Called with g_dev[dev].mu held.
int scratch_ptr(int dev, void** out)
{
    DeviceScratch& d = g_dev[dev];
    if (!d.ptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return TJ_E_HIP;
        d.ptr = p;
    }
    *out = d.ptr;
    return TJ_OK;
}

}  // namespace

extern "C" int tj_sort_static(int key_type, const void* keys_in, const int32_t* rids_in, uint64_t n,
                              void* keys_out, int32_t* rids_out, void* stream, tj_stats_t* stats)
{
    uint64_t min_bytes = 0, full_bytes = 0;
    const int q = tj_workspace_query(TJ_OP_SORT, key_type, n, 0, &min_bytes, &full_bytes);
    if (q != TJ_OK) return q;
    if (min_bytes > TJ_STATIC_SCRATCH_BYTES) return TJ_E_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return TJ_E_HIP;
    if (dev >= kMaxDevices) return TJ_E_ARG;
    try {
        std::lock_guard<std::mutex> g(g_dev[dev].mu);
        void* ws = nullptr;
        const int rc = scratch_ptr(dev, &ws);
        if (rc != TJ_OK) return rc;
        return tj::sort_noalloc(key_type, keys_in, rids_in, n, keys_out, rids_out, ws, TJ_STATIC_SCRATCH_BYTES,
                                stream, stats);
    } catch (...) {
        return TJ_E_INTERNAL;
    }
}

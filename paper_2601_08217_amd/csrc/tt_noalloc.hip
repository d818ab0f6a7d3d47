// Device scratch for the entry point that allocates nothing
// (tt_channel_apply_ul_noalloc): the UL group partials of a call live in one
// file-scope device array instead of memory the library allocates.  Every
// device the library runs on holds its own copy of the array, at its own
// address, until the process ends.
#include "tt_internal.h"

#include <mutex>

namespace {

constexpr int kScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[tt::kNoallocScratchBytes];

std::mutex g_mu;
void* g_ptr[kScratchDevices] = {};

}  // namespace

namespace tt {

// Resolves the array's address on `device` once (with that device current)
// and keeps it; host code uses this address, never the array's name.
hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kScratchDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device])
        return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != device)
        e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess)
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != device)
        (void)hipSetDevice(cur);
    if (e == hipSuccess)
        g_ptr[device] = p;
    return e;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= kScratchDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace tt

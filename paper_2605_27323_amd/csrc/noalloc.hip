// Device memory of the allocation-free render entry point
// (pt_render_frame_noalloc): one file-scope array that each GPU holds for
// the life of the process, reached from the host only through its device
// address.  The array's name in host code is a host-side stand-in, not a
// device address; every host use goes through the address kept here.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace ptmi {

namespace {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_ptr[kNoAllocMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch_init(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ptr[device]) return hipSuccess;
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    e = hipSetDevice(device);
    if (e != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t r = hipSetDevice(prev);
    if (e != hipSuccess) return e;
    if (r != hipSuccess) return r;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
    return hipSuccess;
}

void* noalloc_scratch(int device) {
    if (device < 0 || device >= kNoAllocMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_ptr[device];
}

}  // namespace ptmi

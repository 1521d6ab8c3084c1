// The library's own device scratch memory (noalloc.hip), used by the
// allocation-free render entry point.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace ptmi {

// bytes of the scratch array each GPU holds (counters, work counters and the
// traversal stack overflow area of one megakernel frame)
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;

// Look up and keep the device address of `device`'s copy of the array
// (once per device; makes the device current for the lookup and restores
// the previous one).
hipError_t noalloc_scratch_init(int device);
// The kept address, or nullptr if noalloc_scratch_init has not succeeded
// for this device.
void* noalloc_scratch(int device);

}  // namespace ptmi

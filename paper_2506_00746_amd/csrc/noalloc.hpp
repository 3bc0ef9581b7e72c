// Host interface of the library-owned scratch array (noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace feod {

// Size of the per-device scratch array: 32 MiB, enough for the FP64 E-vector
// of about four million element-node entries (e.g. 32^3 Q3, 48^3 Q2, 16^3 Q7).
constexpr size_t kNoallocScratchBytes = size_t(32) << 20;

// Look up the device address of the scratch array on `device`, which must be
// the current device; done once per device (later calls return at once).
hipError_t noalloc_init(int device);

// The device address found by noalloc_init for `device`, or nullptr.
void* noalloc_scratch(int device);

}  // namespace feod

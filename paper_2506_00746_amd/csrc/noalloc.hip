// Library-owned scratch for the entry points that allocate nothing
// (feod_jacobian_apply_noalloc).  The E-vector of the element stage, the only
// per-call device memory of a Jacobian action besides its inputs and outputs,
// lives in a fixed-size file-scope device array instead of the caller's
// workspace.  Each GPU the library runs on holds its own copy of the array
// (kNoallocScratchBytes) until the process ends.
//
// In host code the array's name is only a host-side stand-in: its device
// address on each GPU is looked up once, with that GPU current, by
// hipGetSymbolAddress, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"

namespace feod {

static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};  // device address of scratch, per device (nullptr: not looked up yet)
}  // namespace

hipError_t noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace feod

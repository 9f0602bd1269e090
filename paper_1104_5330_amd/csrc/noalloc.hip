// Fixed device scratch of sp6_step_noalloc: the RK4 step's T, stage and
// accumulator buffers for callers that cannot allocate device memory.  The
// array is a file-scope device variable, so each GPU holds its own copy (at its
// own address) for as long as the library is loaded.  Host code never uses the
// array's name as an address: it asks the runtime for the device address once
// per device and keeps that pointer.
#include <map>
#include <mutex>

#include "sp6_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[SP6_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
std::map<int, void*> g_ptr;  // device ordinal -> device address of scratch

}  // namespace

// Device address of the scratch on `device`, which must be the current device;
// looked up on the first call per device and cached.
hipError_t noalloc_scratch_ptr(int device, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_ptr.find(device);
  if (it != g_ptr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (p == nullptr) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  *out = p;
  return hipSuccess;
}

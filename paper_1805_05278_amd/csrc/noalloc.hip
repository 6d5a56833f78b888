// Workspace for the entry point that allocates nothing (qr_factor_noalloc):
// a file-scope device array, one copy per GPU, held until the process ends.
// Host code never names the array except to ask the runtime for its address
// on each device (its name on the host is only a stand-in for the symbol).
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace miqr {

static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {
std::mutex g_mu;
double* g_ptr[kNoallocMaxDevices] = {};
}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_ptr[device]) return hipSuccess;
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if (prev != device) e = hipSetDevice(device);
  void* p = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && !p) e = hipErrorInvalidSymbol;
  if (e == hipSuccess) g_ptr[device] = static_cast<double*>(p);
  if (prev != device) (void)hipSetDevice(prev);
  return e;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kNoallocMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_mu);
  return g_ptr[device];
}

}  // namespace miqr

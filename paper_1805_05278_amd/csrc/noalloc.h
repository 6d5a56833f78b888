// The static device workspace of qr_factor_noalloc.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miqr {

// 64 MiB per device.
constexpr int64_t kNoallocDoubles = int64_t(8) << 20;
constexpr int kNoallocMaxDevices = 64;

// Look up the array's address on `device` (made current for the call) once
// and keep it; later calls return at once.
hipError_t noalloc_setup(int device);

// The array's address on `device` (null before noalloc_setup succeeded).
double* noalloc_scratch(int device);

}  // namespace miqr

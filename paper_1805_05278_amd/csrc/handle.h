// The library handle (opaque to callers; shared by the C ABI translation units).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "batched.h"
#include "miqr.h"
#include "profiler.h"

struct miqr_ctx {
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int* dflag = nullptr;
  std::string err;
  double gemm_flops = 0.0;  // multiply-add flops of the GEMMs launched by the last call
  bool profiling = false;
  miqr::KernelTimer timer;
  std::vector<std::string> prof_names;
  // Pinned staging for batched task tables and statuses; table_ev marks the
  // last upload out of it, so the next call may rewrite it.
  miqr::BatchHeader* pin_tasks = nullptr;
  int32_t* pin_status = nullptr;
  int64_t pin_cap = 0;
  hipEvent_t table_ev = nullptr;
};

// Per-kernel HIP-event timing of library launches.  When a handle has
// profiling enabled, every launch site brackets its kernel with two events on
// the launch stream and records the kernel's algorithmic bytes and flops;
// totals per kernel name are read back through the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

namespace miqr {

struct KernelTotals {
  double ms = 0.0;
  int64_t launches = 0;
  double bytes = 0.0;  // algorithmic HBM bytes
  double flops = 0.0;  // algorithmic flops
};

class KernelTimer {
 public:
  ~KernelTimer();
  // Returns a token for end(), or -1 if no event could be created.
  int begin(hipStream_t s, const char* name, double bytes, double flops);
  void end(hipStream_t s, int token);
  // Synchronise pending events and fold them into the totals.
  void collect();
  void clear();
  std::map<std::string, KernelTotals> totals;

 private:
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double bytes, flops;
  };
  hipEvent_t get_event();
  std::vector<Pending> pending_;
  std::vector<hipEvent_t> free_;
};

// The timer of the handle whose entry point is running on this thread (null
// when profiling is off).
extern thread_local KernelTimer* g_timer;

struct TimedLaunch {
  hipStream_t s;
  KernelTimer* timer;
  int token = -1;
  TimedLaunch(hipStream_t s_, const char* name, double bytes, double flops)
      : s(s_), timer(g_timer) {
    if (timer) token = timer->begin(s, name, bytes, flops);
  }
  ~TimedLaunch() {
    if (timer && token >= 0) timer->end(s, token);
  }
};

}  // namespace miqr

#include "profiler.h"

namespace miqr {

thread_local KernelTimer* g_timer = nullptr;

KernelTimer::~KernelTimer() {
  for (auto& p : pending_) {
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  for (auto e : free_) hipEventDestroy(e);
}

hipEvent_t KernelTimer::get_event() {
  if (!free_.empty()) {
    hipEvent_t e = free_.back();
    free_.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int KernelTimer::begin(hipStream_t s, const char* name, double bytes, double flops) {
  Pending p{name, get_event(), get_event(), bytes, flops};
  if (!p.a || !p.b) return -1;
  hipEventRecord(p.a, s);
  pending_.push_back(p);
  return (int)pending_.size() - 1;
}

void KernelTimer::end(hipStream_t s, int token) {
  if (token < 0 || token >= (int)pending_.size()) return;
  hipEventRecord(pending_[token].b, s);
}

void KernelTimer::collect() {
  for (auto& p : pending_) {
    hipEventSynchronize(p.b);
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      KernelTotals& t = totals[p.name];
      t.ms += ms;
      t.launches += 1;
      t.bytes += p.bytes;
      t.flops += p.flops;
    }
    free_.push_back(p.a);
    free_.push_back(p.b);
  }
  pending_.clear();
  (void)hipGetLastError();  // a failed timing query must not surface elsewhere
}

void KernelTimer::clear() {
  collect();
  totals.clear();
}

}  // namespace miqr

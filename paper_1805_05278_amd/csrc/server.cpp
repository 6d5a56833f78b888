// Least-squares serving loop: requests are admitted into device memory under
// an HBM budget, packed into batches, and solved by the persistent batched
// kernel.  Two batches can be in flight: while one computes, the next batch's
// inputs upload on a separate stream, and requests that arrive meanwhile join
// whichever batch launches next (continuous batching).  Each batch is one
// replay of a captured graph (task-table upload, queue reset, persistent
// kernel, status download).  Factorisations can be kept on the device for
// further right-hand sides.
//
// The server is driven by its caller: qr_server_poll retires finished
// batches, admits waiting requests and launches the next batch.  It is not
// thread-safe.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "batched.h"
#include "handle.h"
#include "miqr.h"

using namespace miqr;

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over one device buffer (offsets; coalescing free list).
class Pool {
 public:
  void init(size_t size) {
    size_ = size;
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = round_up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rem = it->second - bytes;
      const size_t o = it->first;
      free_.erase(it);
      if (rem) free_[o + bytes] = rem;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(std::max<size_t>(bytes, 1));
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;
};

enum State { PENDING, ADMITTED, RUNNING, DONE };

struct Buf {
  size_t off = 0, bytes = 0;
  bool live = false;
};

struct Req {
  int64_t id = 0;
  int64_t m = 0, n = 0, nrhs = 0;
  const double* hA = nullptr;
  const double* hB = nullptr;
  double* hX = nullptr;
  int64_t lda = 0, ldb = 0, ldx = 0;
  int64_t parent = -1;  // factored request whose kept factors this one reuses
  bool keep = false;    // keep A (reflector blocks), R and tau after completion
  bool redo = false;    // mixed-precision refinement missed its target: solve in FP64
  State state = PENDING;
  Buf A, B, R, C, tau;
  int ev = -1;          // upload event slot (-1: nothing to wait for)
  int64_t xoff = 0;     // offset (doubles) of its solution in the batch staging
  int status = 0;
  int batch_size = 0;
  double t_submit = 0, t_start = 0, t_end = 0;
};

struct Slot {
  bool busy = false;
  std::vector<int64_t> ids;
  hipEvent_t done = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchHeader* dtable = nullptr;
  BatchHeader* ptable = nullptr;
  int* dstatus = nullptr;
  int32_t* pstatus = nullptr;
  int* dcounter = nullptr;
  double* dx = nullptr;
  double* px = nullptr;
};

}  // namespace

struct miqr_server {
  miqr_handle h = nullptr;
  int64_t max_batch = 4096, max_pending = 1 << 20;
  size_t stage_doubles = 0;
  bool keep = false;
  char* pool_base = nullptr;
  Pool pool;
  hipStream_t compute = nullptr, copy = nullptr;
  Slot slots[2];
  std::vector<hipEvent_t> up_events;
  std::vector<int> up_refs;  // requests still to be launched after each upload event
  int prec = kBlkF64;     // working precision of the batches
  BatchGrids grids{};     // persistent grids for that precision
  BatchGrids grids64{};   // and for FP64 re-solves
  int64_t next_id = 1;
  std::unordered_map<int64_t, Req> reqs;
  std::deque<int64_t> pending;
  std::deque<int64_t> admitted;
  std::deque<qr_server_done> finished;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

miqr_status sfail(miqr_server* s, miqr_status st, const std::string& msg) {
  if (s && s->h) s->h->err = msg;
  return st;
}

miqr_status shfail(miqr_server* s, hipError_t e, const char* where) {
  return sfail(s, MIQR_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

double* dptr(miqr_server* s, const Buf& b) { return (double*)(s->pool_base + b.off); }

int64_t blocks_of(int64_t m) { return (m + kBatchRows - 1) / kBatchRows; }

// Device bytes a request needs at admission.
void sizes(const miqr_server* s, const Req& r, size_t* a, size_t* b, size_t* rr, size_t* c,
           size_t* tau) {
  const bool apply = r.parent >= 0;
  *a = apply ? 0 : (size_t)(r.m * r.n) * 8;
  *b = (size_t)(r.m * r.nrhs) * 8;
  *rr = apply ? 0 : (size_t)(r.n * r.n) * 8;
  *c = (size_t)(r.n * r.nrhs) * 8;
  *tau = (!apply && r.keep) ? (size_t)(blocks_of(r.m) * r.n) * 8 : 0;
  (void)s;
}

void free_buf(miqr_server* s, Buf& b) {
  if (b.live) s->pool.release(b.off, b.bytes);
  b.live = false;
}

bool alloc_buf(miqr_server* s, Buf& b, size_t bytes) {
  b.bytes = bytes;
  b.live = false;
  if (bytes == 0) return true;
  if (!s->pool.alloc(bytes, &b.off)) return false;
  b.live = true;
  return true;
}

int take_event(miqr_server* s) {
  for (size_t i = 0; i < s->up_events.size(); ++i)
    if (s->up_refs[i] == 0) return (int)i;
  hipEvent_t e;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return -1;
  s->up_events.push_back(e);
  s->up_refs.push_back(0);
  return (int)s->up_events.size() - 1;
}

// Move waiting requests into device memory while the budget allows (in
// arrival order; the first one that does not fit waits, and so do the rest).
miqr_status admit(miqr_server* s) {
  int ev = -1;
  while (!s->pending.empty()) {
    Req& r = s->reqs[s->pending.front()];
    size_t a, b, rr, c, tau;
    sizes(s, r, &a, &b, &rr, &c, &tau);
    if (!alloc_buf(s, r.A, a)) break;
    if (!alloc_buf(s, r.B, b)) {
      free_buf(s, r.A);
      break;
    }
    if (!alloc_buf(s, r.R, rr) || !alloc_buf(s, r.C, c) || !alloc_buf(s, r.tau, tau)) {
      free_buf(s, r.A);
      free_buf(s, r.B);
      free_buf(s, r.R);
      free_buf(s, r.C);
      free_buf(s, r.tau);
      break;
    }
    hipError_t e = hipSuccess;
    if (a)
      e = hipMemcpy2DAsync(dptr(s, r.A), (size_t)r.m * 8, r.hA, (size_t)r.lda * 8,
                           (size_t)r.m * 8, (size_t)r.n, hipMemcpyHostToDevice, s->copy);
    if (e == hipSuccess)
      e = hipMemcpy2DAsync(dptr(s, r.B), (size_t)r.m * 8, r.hB, (size_t)r.ldb * 8,
                           (size_t)r.m * 8, (size_t)r.nrhs, hipMemcpyHostToDevice, s->copy);
    if (e != hipSuccess) return shfail(s, e, "server upload");
    if (ev < 0) {
      ev = take_event(s);
      if (ev < 0) return sfail(s, MIQR_EHIP, "server: event creation failed");
    }
    r.ev = ev;
    s->up_refs[ev]++;
    r.state = ADMITTED;
    s->admitted.push_back(r.id);
    s->pending.pop_front();
  }
  if (ev >= 0) {
    hipError_t e = hipEventRecord(s->up_events[ev], s->copy);
    if (e != hipSuccess) return shfail(s, e, "server upload event");
  }
  return MIQR_OK;
}

// Launch the next batch on slot sl.  A batch is either requests in the
// server's precision (one replay of the slot's graph) or FP64 re-solves of
// mixed-precision requests whose refinement missed its target (the same
// sequence launched directly).  Tasks are grouped by queue of the batched
// kernels, largest first within a queue.
miqr_status launch(miqr_server* s, Slot& sl) {
  const bool redo = s->reqs[s->admitted.front()].redo;
  int count = 0;
  int64_t xoff = 0;
  std::vector<int> evs;
  std::vector<BatchTask> tk;
  sl.ids.clear();
  while (!s->admitted.empty() && count < s->max_batch) {
    Req& r = s->reqs[s->admitted.front()];
    if (r.redo != redo) break;
    const int64_t xs = r.n * r.nrhs;
    if (xoff + xs > (int64_t)s->stage_doubles) break;
    BatchTask t{};
    if (r.parent >= 0) {
      const Req& p = s->reqs[r.parent];
      t.A = dptr(s, p.A);
      t.R = dptr(s, p.R);
      t.tau = dptr(s, p.tau);
      t.flags = kTaskApply;
    } else {
      t.A = dptr(s, r.A);
      t.R = dptr(s, r.R);
      t.tau = r.keep ? dptr(s, r.tau) : nullptr;
      t.flags = r.keep ? kTaskKeep : 0;
    }
    t.B = dptr(s, r.B);
    t.C = dptr(s, r.C);
    t.X = sl.dx + xoff;
    t.lda = r.m;
    t.ldb = r.m;
    t.m = (int)r.m;
    t.n = (int)r.n;
    t.nrhs = (int)r.nrhs;
    t.slot = count++;
    tk.push_back(t);
    r.xoff = xoff;
    xoff += (xs + 31) & ~int64_t(31);
    r.state = RUNNING;
    if (r.ev >= 0 && std::find(evs.begin(), evs.end(), r.ev) == evs.end()) evs.push_back(r.ev);
    sl.ids.push_back(r.id);
    s->admitted.pop_front();
  }
  if (count == 0) return MIQR_OK;
  std::vector<int> q(tk.size());
  std::vector<size_t> order(tk.size());
  for (size_t k = 0; k < tk.size(); ++k) {
    q[k] = batch_queue(tk[k]);
    order[k] = k;
  }
  auto cost = [&](size_t k) {
    const double N = (double)tk[k].n + tk[k].nrhs;
    return ((tk[k].m + kBatchRows - 1) / kBatchRows + 1) * N * N;
  };
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return q[a] != q[b] ? q[a] < q[b] : cost(a) > cost(b);
  });
  BatchHeader* hd = sl.ptable;
  *hd = BatchHeader{};
  hd->total = count;
  BatchTask* tasks = batch_tasks(hd);
  for (size_t k = 0; k < order.size(); ++k) {
    tasks[k] = tk[order[k]];
    hd->count[q[order[k]]]++;
  }
  for (int k = 1; k < kBatchQueues; ++k) hd->begin[k] = hd->begin[k - 1] + hd->count[k - 1];
  hipError_t e = hipSuccess;
  for (int ev : evs) {
    if (e == hipSuccess) e = hipStreamWaitEvent(s->compute, s->up_events[ev], 0);
  }
  for (int64_t id : sl.ids) {
    Req& r = s->reqs[id];
    if (r.ev >= 0) s->up_refs[r.ev]--;
    r.ev = -1;
  }
  if (!redo) {
    if (e == hipSuccess) e = hipGraphLaunch(sl.exec, s->compute);
  } else {
    const size_t tb = batch_table_bytes(count);
    if (e == hipSuccess) e = hipMemcpyAsync(sl.dtable, sl.ptable, tb, hipMemcpyHostToDevice, s->compute);
    if (e == hipSuccess) {
      batched_ls(s->compute, sl.dtable, sl.dcounter, sl.dstatus, nullptr, s->grids64, kBlkF64, 0.0,
                 0.0);
      e = hipGetLastError();
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(sl.pstatus, sl.dstatus, (size_t)count * 4, hipMemcpyDeviceToHost,
                         s->compute);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.px, sl.dx, (size_t)xoff * 8, hipMemcpyDeviceToHost, s->compute);
  if (e == hipSuccess) e = hipEventRecord(sl.done, s->compute);
  if (e != hipSuccess) return shfail(s, e, "server launch");
  const double t = s->now();
  for (int64_t id : sl.ids) {
    Req& r = s->reqs[id];
    if (!r.redo) r.t_start = t;
    r.batch_size = count;
  }
  sl.busy = true;
  return MIQR_OK;
}

void retire(miqr_server* s, Slot& sl) {
  const double t = s->now();
  std::vector<int64_t> again;
  for (size_t k = 0; k < sl.ids.size(); ++k) {
    const int64_t id = sl.ids[k];
    Req& r = s->reqs[id];
    r.status = sl.pstatus[k];
    if (r.status == kStatusNoConv) {
      // A and B are on the device as uploaded: solve again in FP64.
      r.redo = true;
      r.state = ADMITTED;
      again.push_back(id);
      continue;
    }
    const double* src = sl.px + r.xoff;
    for (int64_t k = 0; k < r.nrhs; ++k)
      std::memcpy(r.hX + k * r.ldx, src + k * r.n, (size_t)r.n * 8);
    r.t_end = t;
    r.state = DONE;
    free_buf(s, r.B);
    free_buf(s, r.C);
    if (!r.keep) {
      free_buf(s, r.A);
      free_buf(s, r.R);
      free_buf(s, r.tau);
    }
    qr_server_done d{};
    d.id = r.id;
    d.status = r.status;
    d.batch_size = r.batch_size;
    d.submit_s = r.t_submit;
    d.start_s = r.t_start;
    d.end_s = r.t_end;
    s->finished.push_back(d);
    if (!r.keep) s->reqs.erase(id);
  }
  for (auto it = again.rbegin(); it != again.rend(); ++it) s->admitted.push_front(*it);
  sl.ids.clear();
  sl.busy = false;
}

// Retire finished batches (blocking on the oldest one if `block`).
miqr_status reap(miqr_server* s, bool block) {
  for (int pass = 0; pass < 2; ++pass) {
    Slot* oldest = nullptr;
    for (Slot& sl : s->slots)
      if (sl.busy && (!oldest || sl.ids.front() < oldest->ids.front())) oldest = &sl;
    if (!oldest) return MIQR_OK;
    hipError_t e = block ? hipEventSynchronize(oldest->done) : hipEventQuery(oldest->done);
    if (e == hipErrorNotReady) return MIQR_OK;
    if (e != hipSuccess) return shfail(s, e, "server batch");
    retire(s, *oldest);
    block = false;
  }
  return MIQR_OK;
}

miqr_status make_slot(miqr_server* s, Slot& sl) {
  hipError_t e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
  const size_t tb = batch_table_bytes(s->max_batch);
  if (e == hipSuccess) e = hipMalloc((void**)&sl.dtable, tb);
  if (e == hipSuccess) e = hipMalloc((void**)&sl.dstatus, (size_t)s->max_batch * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&sl.dcounter, 256);
  if (e == hipSuccess) e = hipMalloc((void**)&sl.dx, s->stage_doubles * 8);
  if (e == hipSuccess) e = hipHostMalloc((void**)&sl.ptable, tb, hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&sl.pstatus, (size_t)s->max_batch * 4, hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void**)&sl.px, s->stage_doubles * 8, hipHostMallocDefault);
  if (e != hipSuccess) return sfail(s, MIQR_ENOMEM, "server: slot allocation failed");
  std::memset(sl.ptable, 0, tb);
  // One batch = one replay: table upload, queue reset + persistent kernel,
  // status download.  The table's header carries the count, so the graph
  // never changes.
  e = hipStreamBeginCapture(s->compute, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) e = hipMemcpyAsync(sl.dtable, sl.ptable, tb, hipMemcpyHostToDevice, s->compute);
  if (e == hipSuccess) {
    batched_ls(s->compute, sl.dtable, sl.dcounter, sl.dstatus, nullptr, s->grids, s->prec, 0.0,
               0.0);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(sl.pstatus, sl.dstatus, (size_t)s->max_batch * 4, hipMemcpyDeviceToHost,
                       s->compute);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(s->compute, &g);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&sl.exec, g, nullptr, nullptr, 0);
  sl.graph = g;
  if (e != hipSuccess) return shfail(s, e, "server graph capture");
  return MIQR_OK;
}

void destroy_server(miqr_server* s) {
  if (s->compute) hipStreamSynchronize(s->compute);
  if (s->copy) hipStreamSynchronize(s->copy);
  for (Slot& sl : s->slots) {
    if (sl.exec) hipGraphExecDestroy(sl.exec);
    if (sl.graph) hipGraphDestroy(sl.graph);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.dtable) hipFree(sl.dtable);
    if (sl.dstatus) hipFree(sl.dstatus);
    if (sl.dcounter) hipFree(sl.dcounter);
    if (sl.dx) hipFree(sl.dx);
    if (sl.ptable) hipHostFree(sl.ptable);
    if (sl.pstatus) hipHostFree(sl.pstatus);
    if (sl.px) hipHostFree(sl.px);
  }
  for (hipEvent_t e : s->up_events) hipEventDestroy(e);
  if (s->pool_base) hipFree(s->pool_base);
  if (s->compute) hipStreamDestroy(s->compute);
  if (s->copy) hipStreamDestroy(s->copy);
  delete s;
}

miqr_status check_host(const void* p, int64_t ld, int64_t rows) {
  return (p && ld >= rows) ? MIQR_OK : MIQR_EINVAL;
}

}  // namespace

extern "C" {

miqr_status qr_server_create(miqr_handle h, const qr_server_opts* o, miqr_server_handle* out) {
  if (!h || !out) return MIQR_EINVAL;
  *out = nullptr;
  h->err.clear();
  const int64_t budget = (o && o->hbm_budget > 0) ? o->hbm_budget : (int64_t)8 << 30;
  const int64_t maxb = (o && o->max_batch > 0) ? o->max_batch : 4096;
  const int64_t stage = (o && o->stage_bytes > 0) ? o->stage_bytes : (int64_t)64 << 20;
  if (maxb > (1 << 20)) {
    h->err = "max_batch above 2^20";
    return MIQR_EINVAL;
  }
  if (stage < (int64_t)kBatchMaxCols * kBatchMaxCols * 2) {
    h->err = "stage_bytes too small for one request";
    return MIQR_EINVAL;
  }
  const int prec = o ? o->precision : MIQR_FP64;
  if (prec != MIQR_FP64 && prec != MIQR_MIXED_FP32 && prec != MIQR_MIXED_BF16) {
    h->err = "unknown precision";
    return MIQR_EINVAL;
  }
  if (prec != MIQR_FP64 && o->keep_factors) {
    // Kept factors are replayed on later right-hand sides without
    // refinement, so they are FP64 only.
    h->err = "keep_factors needs precision MIQR_FP64";
    return MIQR_ENOTSUP;
  }
  if (hipSetDevice(h->device) != hipSuccess) return MIQR_EHIP;
  miqr_server* s = new miqr_server();
  s->h = h;
  s->max_batch = maxb;
  s->max_pending = (o && o->max_pending > 0) ? o->max_pending : (int64_t)1 << 20;
  s->stage_doubles = (size_t)stage / 8;
  s->keep = o && o->keep_factors;
  s->t0 = std::chrono::steady_clock::now();
  s->prec = prec == MIQR_MIXED_FP32 ? kBlkF32 : (prec == MIQR_MIXED_BF16 ? kBlkBF16 : kBlkF64);
  s->grids = batched_grids(h->device, s->prec);
  s->grids64 = batched_grids(h->device, kBlkF64);
  hipError_t e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
  if (e != hipSuccess) {
    destroy_server(s);
    return MIQR_EHIP;
  }
  if (hipMalloc((void**)&s->pool_base, (size_t)budget) != hipSuccess) {
    (void)hipGetLastError();
    destroy_server(s);
    h->err = "server: HBM budget allocation failed";
    return MIQR_ENOMEM;
  }
  s->pool.init((size_t)budget);
  for (Slot& sl : s->slots) {
    miqr_status st = make_slot(s, sl);
    if (st != MIQR_OK) {
      destroy_server(s);
      return st;
    }
  }
  *out = s;
  return MIQR_OK;
}

miqr_status qr_server_destroy(miqr_server_handle s) {
  if (!s) return MIQR_EINVAL;
  hipSetDevice(s->h->device);
  destroy_server(s);
  return MIQR_OK;
}

double qr_server_clock(miqr_server_handle s) { return s ? s->now() : 0.0; }

miqr_status qr_server_submit(miqr_server_handle s, int64_t m, int64_t n, int64_t nrhs,
                             const double* A, int64_t lda, const double* B, int64_t ldb,
                             double* X, int64_t ldx, int64_t* id) {
  if (!s || !id) return MIQR_EINVAL;
  s->h->err.clear();
  if (n < 1 || m < n || m > INT32_MAX) return sfail(s, MIQR_EINVAL, "need 2^31 > m >= n >= 1");
  if (nrhs < 1 || nrhs > kBatchMaxRhs || n + nrhs > kBatchMaxCols)
    return sfail(s, MIQR_EINVAL, "need 1 <= nrhs <= 8 and n + nrhs <= 320");
  if (check_host(A, lda, m) || check_host(B, ldb, m) || check_host(X, ldx, n))
    return sfail(s, MIQR_EINVAL, "null pointer or leading dimension too small");
  Req r;
  r.m = m;
  r.n = n;
  r.nrhs = nrhs;
  r.hA = A;
  r.hB = B;
  r.hX = X;
  r.lda = lda;
  r.ldb = ldb;
  r.ldx = ldx;
  r.keep = s->keep;
  size_t a, b, rr, c, tau;
  sizes(s, r, &a, &b, &rr, &c, &tau);
  if (round_up(a) + round_up(b) + round_up(rr) + round_up(c) + round_up(tau) > s->pool.size())
    return sfail(s, MIQR_EINVAL, "request larger than the server's HBM budget");
  if ((int64_t)s->pending.size() >= s->max_pending)
    return sfail(s, MIQR_EBUSY, "too many requests waiting for admission");
  r.id = s->next_id++;
  r.t_submit = s->now();
  *id = r.id;
  s->reqs[r.id] = r;
  s->pending.push_back(r.id);
  return MIQR_OK;
}

miqr_status qr_server_resolve(miqr_server_handle s, int64_t factored, int64_t nrhs,
                              const double* B, int64_t ldb, double* X, int64_t ldx, int64_t* id) {
  if (!s || !id) return MIQR_EINVAL;
  s->h->err.clear();
  auto it = s->reqs.find(factored);
  if (it == s->reqs.end() || !it->second.keep || it->second.parent >= 0)
    return sfail(s, MIQR_EINVAL, "no kept factorisation with that id");
  const Req& p = it->second;
  if (p.state != DONE) return sfail(s, MIQR_EBUSY, "factorisation not finished yet");
  if (p.status != 0) return sfail(s, MIQR_ESINGULAR, "kept factorisation is singular");
  if (nrhs < 1 || nrhs > kBatchMaxRhs || p.n + nrhs > kBatchMaxCols)
    return sfail(s, MIQR_EINVAL, "need 1 <= nrhs <= 8 and n + nrhs <= 320");
  if (check_host(B, ldb, p.m) || check_host(X, ldx, p.n))
    return sfail(s, MIQR_EINVAL, "null pointer or leading dimension too small");
  if ((int64_t)s->pending.size() >= s->max_pending)
    return sfail(s, MIQR_EBUSY, "too many requests waiting for admission");
  Req r;
  r.m = p.m;
  r.n = p.n;
  r.nrhs = nrhs;
  r.hB = B;
  r.hX = X;
  r.ldb = ldb;
  r.ldx = ldx;
  r.parent = factored;
  r.id = s->next_id++;
  r.t_submit = s->now();
  *id = r.id;
  s->reqs[r.id] = r;
  s->pending.push_back(r.id);
  return MIQR_OK;
}

miqr_status qr_server_release(miqr_server_handle s, int64_t factored) {
  if (!s) return MIQR_EINVAL;
  auto it = s->reqs.find(factored);
  if (it == s->reqs.end() || !it->second.keep || it->second.parent >= 0)
    return sfail(s, MIQR_EINVAL, "no kept factorisation with that id");
  if (it->second.state != DONE) return sfail(s, MIQR_EBUSY, "factorisation not finished yet");
  for (const auto& kv : s->reqs)
    if (kv.second.parent == factored && kv.second.state != DONE)
      return sfail(s, MIQR_EBUSY, "right-hand sides still in flight on this factorisation");
  Req& r = it->second;
  free_buf(s, r.A);
  free_buf(s, r.R);
  free_buf(s, r.tau);
  // Finished solves against it no longer need their record.
  for (auto jt = s->reqs.begin(); jt != s->reqs.end();) {
    if (jt->second.parent == factored) jt = s->reqs.erase(jt);
    else ++jt;
  }
  s->reqs.erase(factored);
  return MIQR_OK;
}

miqr_status qr_server_poll(miqr_server_handle s, int wait, qr_server_done* done, int64_t cap,
                           int64_t* ndone) {
  if (!s || !ndone || cap < 0 || (cap > 0 && !done)) return MIQR_EINVAL;
  s->h->err.clear();
  *ndone = 0;
  if (hipSetDevice(s->h->device) != hipSuccess) return MIQR_EHIP;
  miqr_status st = reap(s, false);
  if (st == MIQR_OK) st = admit(s);
  for (Slot& sl : s->slots)
    if (st == MIQR_OK && !sl.busy && !s->admitted.empty()) st = launch(s, sl);
  if (st != MIQR_OK) return st;
  if (wait && s->finished.empty()) {
    st = reap(s, true);
    if (st == MIQR_OK) st = admit(s);
    for (Slot& sl : s->slots)
      if (st == MIQR_OK && !sl.busy && !s->admitted.empty()) st = launch(s, sl);
    if (st != MIQR_OK) return st;
  }
  while (*ndone < cap && !s->finished.empty()) {
    done[(*ndone)++] = s->finished.front();
    s->finished.pop_front();
  }
  return MIQR_OK;
}

miqr_status qr_server_stats(miqr_server_handle s, int64_t* pending, int64_t* admitted,
                            int64_t* running, int64_t* hbm_used) {
  if (!s) return MIQR_EINVAL;
  int64_t run = 0;
  for (const Slot& sl : s->slots) run += sl.busy ? (int64_t)sl.ids.size() : 0;
  if (pending) *pending = (int64_t)s->pending.size();
  if (admitted) *admitted = (int64_t)s->admitted.size();
  if (running) *running = run;
  if (hbm_used) *hbm_used = (int64_t)s->pool.used();
  return MIQR_OK;
}

}  // extern "C"

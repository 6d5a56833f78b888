// The library handle (opaque to callers; shared by the C ABI translation units).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include <map>
#include <tuple>

#include "batched.h"
#include "miqr.h"
#include "plan.h"
#include "profiler.h"

// Key of the handle's tuning cache: the shape and every option the cost model
// reads.
struct TuneKey {
  int64_t m, n, lstsq, b, bstar, nb, leaf_rows, chain, arity, layout, nola;
  bool operator<(const TuneKey& o) const {
    return std::tie(m, n, lstsq, b, bstar, nb, leaf_rows, chain, arity, layout, nola) <
           std::tie(o.m, o.n, o.lstsq, o.b, o.bstar, o.nb, o.leaf_rows, o.chain, o.arity,
                    o.layout, o.nola);
  }
};

// Key of the handle's factorisation graphs: everything a captured launch
// sequence bakes in (shape, leading dimensions, buffer addresses, options and
// the resolved tuning).
struct GraphKey {
  int64_t m, n, lda, ldt, ldq;
  const void *A, *T, *Q, *sign, *ws;
  int64_t normalize, prec, b, bstar, nb, leaf_rows, chain, arity, layout, lookahead;
  bool operator<(const GraphKey& o) const {
    return std::tie(m, n, lda, ldt, ldq, A, T, Q, sign, ws, normalize, prec, b, bstar, nb,
                    leaf_rows, chain, arity, layout, lookahead) <
           std::tie(o.m, o.n, o.lda, o.ldt, o.ldq, o.A, o.T, o.Q, o.sign, o.ws, o.normalize,
                    o.prec, o.b, o.bstar, o.nb, o.leaf_rows, o.chain, o.arity, o.layout,
                    o.lookahead);
  }
};
struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  double gemm_flops = 0.0;
};

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
  // Look-ahead of the right-looking top level: a second stream (default
  // priority) and the two events that order it against the caller's stream.
  hipStream_t aux = nullptr;
  hipEvent_t ev_panel = nullptr;
  hipEvent_t ev_update = nullptr;
  std::map<TuneKey, miqr::Tuning> tune_cache;
  // qr_factor launch sequences captured once and replayed (miqr_graphs_enable);
  // cap is the stream they are captured on (never executed on).
  bool graphs = false;
  hipStream_t cap = nullptr;
  std::map<GraphKey, GraphEntry> graph_cache;
};

// TSQR panel factorisation (base case of the EG recursion): host interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

#include "common.h"

namespace miqr {

// One level of the TSQR reduction.  Level 0 holds the leaf row blocks of the
// panel; level l > 0 holds the R factors produced by the chains of level l-1.
// Consecutive blocks of a level are grouped into chains of `chain_len` blocks
// that one workgroup reduces in sequence.
struct TsqrLevel {
  int nblocks = 0;
  int chain_len = 1;
  int nchains = 0;
  double* T = nullptr;  // per block, kTS doubles each
  double* Y = nullptr;  // per block (levels > 0 only), kTS doubles each
  double* R = nullptr;  // per chain, kTS doubles each
  double* B = nullptr;  // per chain, downsweep input, kBS doubles each
};

struct TsqrPlan {
  int64_t rows = 0;    // panel rows
  int nbr = 0;         // panel width (<= kNB)
  int leaf_rows = 0;   // 128 or 256
  std::vector<TsqrLevel> levels;
  double* LR = nullptr;  // kTS doubles: final L (strict lower) and R of the top rows
  int64_t workspace_doubles = 0;
};

// Choose block sizes and lay the plan's arrays out in `ws` (may be null to
// only compute the size).
TsqrPlan tsqr_plan(int64_t rows, int nbr, int leaf_rows, int chain, int arity, double* ws);

// Factor the rows x nbr panel at P (leading dimension ldp) in place:
// V below the diagonal, R on and above it; the nbr x nbr kernel T into Tp
// (ldt).  Optional: explicit thin Q (ldq), with columns scaled by D when
// `normalize` (then R holds D R and `sign` receives D).
hipError_t tsqr_factor(const TsqrPlan& plan, hipStream_t s, double* P, int64_t ldp,
                       double* Tp, int64_t ldt, double* Q, int64_t ldq, int normalize,
                       double* sign);

}  // namespace miqr

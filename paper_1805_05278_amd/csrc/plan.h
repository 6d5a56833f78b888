// Host-side planning of one factorisation: the tuning (what the paper leaves
// as tunable parameters: the recursion threshold b and base-case width b* of
// Sec. 6.3 and Sec. 7.3, the TSQR block height and tree shape of App. C, the
// right-looking top level of Sec. 8.4), the Alg. 2 split rule, the workspace
// layout, and the cost model that chooses the tuning (Sec. 3: time =
// alpha * launches + beta * bytes + gamma * flops, with the paper's messages
// mapped to dependent kernel launches on one GPU).
#pragma once
#include <stdint.h>

#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "miqr.h"

namespace miqr {

enum TLayout : int { T_FULL = MIQR_T_FULL, T_BLOCKED = MIQR_T_BLOCKED };

// Largest EG threshold and top-level panel width accepted.
constexpr int64_t kMaxB = 4096;
constexpr int64_t kMaxNB = 4096;

struct Tuning {
  int64_t b = 64;       // Alg. 2 threshold: nodes at most b wide are base cases
  int bstar = 64;       // base case (1D-CAQR-EG): TSQR panels at most b* wide
  int64_t nb = 0;       // width of the right-looking top level's panels (BLOCKED)
  int leaf_rows = 0;    // TSQR leaf block height; 0: per panel, by the cost model
  int chain = 0;        // leaf blocks per workgroup chain; 0: per panel
  int arity = 0;        // TSQR tree arity; 0: per panel
  int t_layout = T_FULL;
  int lookahead = 1;    // BLOCKED: factor panel k+1 beside the update of panel k
};

// TSQR geometry of one panel (rows x w) for given (possibly automatic)
// parameters; shared by the planner, the cost model and tsqr_plan.
struct TsqrGeom {
  int leaf_rows = 0, chain = 0, arity = 0;
  int64_t blocks = 0;       // leaf blocks P0
  int64_t chains = 0;       // leaf chains (workgroups of the leaf launches)
  int levels = 0;           // tree levels above the leaf chains
  int64_t tree_nodes = 0;   // nodes over all tree levels
};
TsqrGeom tsqr_geometry(int64_t rows, int w, int leaf_rows, int chain, int arity);

// Split of an Alg. 2 node of width nk under tuning t: the left width n1, or 0
// for a base case.  Above b the split is ceil(nk / 2) rounded up to a multiple
// of b; between b* and b (inside the base case, 1D-CAQR-EG) to a multiple of
// b*.  Any split gives the same factors in exact arithmetic.
int64_t eg_split(int64_t nk, const Tuning& t);

// Workspace regions of one factorisation, in doubles, in this order.
struct FactorLayout {
  int64_t tsqr = 0;     // TSQR plan of the largest panel
  int64_t wa = 0;       // Alg. 2 temporaries M1 / M3 (largest n1 x n2 of any node)
  int64_t wb = 0;       // M2 / M4
  int64_t scratch = 0;  // split-K partials of the main stream's products
  int64_t u1 = 0;       // top-level update V^T C (BLOCKED)
  int64_t u2 = 0;       // T^T (V^T C)
  int64_t ua1 = 0;      // the same for the look-ahead stream
  int64_t ua2 = 0;
  int64_t scratch_aux = 0;
  int64_t total = 0;
};
// with_q: room for forming the explicit thin Q after the factorisation.
FactorLayout factor_layout(int64_t m, int64_t n, const Tuning& t, bool with_q = false);

// The cost model is linear in its coefficients: a factorisation's time on one
// stream is sum_i coef_i * feature_i over these counts (the paper's
// alpha S + beta W + gamma F of Sec. 3, with S split by the kind of launch,
// since each kind has its own latency on one GPU).
enum CostFeature : int {
  F_LEAF256 = 0,  // serial block-QR steps of 256-row leaves (per launch wave)
  F_LEAF128,      // the same at 128-row leaves
  F_TREE,         // tree levels on the blocked node kernel (> 128 stacked rows)
  F_TREE_SMALL,   // tree levels on the column-by-column node kernel
  F_HR,           // Householder reconstructions (one per TSQR panel)
  F_DOWN,         // downsweep levels (tree levels + the leaf level)
  F_GEMM_LAUNCH,  // GEMM and split-K reduce launches
  F_GEMM_FLOP,    // GEMM flops
  F_GEMM_DEPTH,   // GEMM flops / d, d the product's smallest dimension (short
                  // products pay their tile prologue and epilogue more often)
  F_GEMM_IDLE,    // GEMM flops * (256 / workgroups - 1) for products with
                  // fewer workgroups than CUs
  F_BYTES,        // algorithmic HBM bytes of the TSQR kernels
  F_COUNT
};
const char* cost_feature_name(int f);

// Coefficients (seconds per count; F_GEMM_FLOP: seconds per flop, the
// inverse of the asymptotic FP64 MFMA rate; F_GEMM_DEPTH: that times the
// depth d0 at which a product runs at half its asymptotic rate; F_BYTES: the
// inverse of the panel kernels' bandwidth) and the look-ahead overlap: the
// share of the shorter of the two concurrent streams that still adds to the
// time.
struct CostCoeffs {
  double c[F_COUNT];
  double overlap;
};
const CostCoeffs& cost_coeffs();

// Features of one top-level panel of a BLOCKED factorisation: its own
// factorisation, the update of the next panel's columns, the rest of the
// update.
struct PanelFeatures {
  double part[3][F_COUNT];
  PanelFeatures(const double* a, const double* b, const double* c) {
    for (int i = 0; i < F_COUNT; ++i) {
      part[0][i] = a[i];
      part[1][i] = b[i];
      part[2][i] = c[i];
    }
  }
};

// What the cost model counts for one factorisation.
struct CostEstimate {
  double seconds = 0.0;
  double f[F_COUNT] = {};    // features summed over the whole factorisation
  int64_t panels = 0;        // TSQR panels
  double gemm_flops = 0.0;   // algorithmic flops of the GEMMs
  double critical_s = 0.0;   // panel factorisations alone
  double update_s = 0.0;     // top-level updates alone (BLOCKED)
  std::vector<PanelFeatures> schedule;  // BLOCKED: per top-level panel
};
CostEstimate predict(int64_t m, int64_t n, const Tuning& t);

// Tuning for a factorisation from the caller's options: fields the caller set
// are kept (after validation by the entry point); the rest are chosen by the
// cost model.  `lstsq` asks for the layout least squares uses.
Tuning choose_tuning(int64_t m, int64_t n, const qr_opts* o, bool lstsq = false);

// TSQR parameters for one panel when the caller left them automatic.
void tsqr_auto(int64_t rows, int w, int* leaf_rows, int* chain, int* arity);

// JSON description of the plan (tuning, cost, workspace regions, recursion
// nodes); host only.
std::string describe_plan(int64_t m, int64_t n, const Tuning& t);

}  // namespace miqr

// The factorisation driver: Alg. 2 (QR-EG) with the TSQR base case, and its
// right-looking top level (Sec. 8.4) with per-panel T and a one-panel
// look-ahead; application and formation of Q in both T layouts.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.h"

namespace miqr {

// Device regions of one factorisation, carved from a workspace in the order
// of FactorLayout (base may be null: only the offsets are computed).
struct FactorWs {
  double* tsqr = nullptr;
  double* wa = nullptr;
  double* wb = nullptr;
  double* scratch = nullptr;
  double* u1 = nullptr;
  double* u2 = nullptr;
  double* ua1 = nullptr;
  double* ua2 = nullptr;
  double* scratch_aux = nullptr;
  int64_t w_cap = 0, scratch_n = 0, u_cap = 0, ua_cap = 0, scratch_aux_n = 0;
  int64_t doubles = 0;  // extent of the carved regions
};
FactorWs carve_factor(double* base, const FactorLayout& L);

// Streams and events of the right-looking top level's look-ahead.
struct Lookahead {
  hipStream_t aux = nullptr;
  hipEvent_t ev_panel = nullptr;   // main: panel k factored
  hipEvent_t ev_update = nullptr;  // aux: update of panel k done
};

struct FactorArgs {
  int64_t m = 0, n = 0;
  double* A = nullptr;
  int64_t lda = 0;
  double* T = nullptr;  // FULL: n x n; BLOCKED: nb x n (panel k's T in columns of panel k)
  int64_t ldt = 0;
  int update_compute = 0;      // arithmetic of the trailing-update products (Compute)
  bool skip_spine_t = false;   // FULL, least squares: leave the right spine's T12 blocks
  double* Q = nullptr;         // optional thin Q
  int64_t ldq = 0;
  int normalize = 0;
  double* sign = nullptr;
};

// Factor A in place on stream s (and la.aux for the look-ahead).  Adds the
// flops of every GEMM launched to *flops.
hipError_t run_factor(hipStream_t s, const Lookahead& la, const Tuning& t, const FactorWs& w,
                      const FactorArgs& a, double* flops);

// C <- Q C ('N') or Q^T C ('T') with the factors of a BLOCKED factorisation:
// panels of width nb, panel k's T in T[0:w_k, k nb : k nb + w_k].  W1, W2 hold
// nb x k doubles each.
hipError_t apply_q_blocked(hipStream_t s, char trans, int64_t m, int64_t n, int64_t k,
                           const double* VR, int64_t lda, const double* T, int64_t ldt, int64_t nb,
                           double* C, int64_t ldc, double* W1, double* W2, double* scratch,
                           int64_t scratch_n);

// C <- Q C or Q^T C with the full n x n T (three products, right to left).
hipError_t apply_q_full(hipStream_t s, char trans, int64_t m, int64_t n, int64_t k,
                        const double* VR, int64_t lda, const double* T, int64_t ldt, double* C,
                        int64_t ldc, double* W1, double* W2, double* scratch, int64_t scratch_n);

// Q^T C for FULL factors whose right-spine T12 blocks were left unassembled:
// Q = Q_L Q_R at every spine node, so (V_L, T_L)^T goes to the node's rows and
// the walk moves to the right child.
hipError_t apply_qt_spine(hipStream_t s, int64_t m, int64_t n, int64_t k, const double* VR,
                          int64_t lda, const double* T, int64_t ldt, double* C, int64_t ldc,
                          const Tuning& t, double* W1, double* W2, double* scratch,
                          int64_t scratch_n);

// Explicit thin Q (m x n, ldq) of BLOCKED factors: [I; 0] with the panels'
// reflectors applied last to first; columns scaled by sign when given.
// W1, W2 hold nb x n doubles each.
hipError_t form_q_blocked(hipStream_t s, int64_t m, int64_t n, const double* VR, int64_t lda,
                          const double* T, int64_t ldt, int64_t nb, const double* sign, double* Q,
                          int64_t ldq, double* W1, double* W2, double* scratch,
                          int64_t scratch_n);

}  // namespace miqr

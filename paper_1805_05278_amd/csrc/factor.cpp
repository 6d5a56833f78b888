// The factorisation driver.  Alg. 2 (QR-EG): split the columns, factor the
// left half, update the right half with C <- C - V_L (T_L^T (V_L^T C)), factor
// the lower right block, assemble T; below the threshold the base case is the
// TSQR panel factorisation (App. C).  With the BLOCKED T layout the top level
// of the recursion is replaced by a right-looking loop over panels (the
// T-avoiding variant of Sec. 8.4): each panel is factored by Alg. 2 and keeps
// its own T, and the trailing matrix is updated panel by panel, so the
// superdiagonal blocks of T between panels are never formed.  Panel k + 1 is
// factored on the caller's stream while a second stream applies panel k to the
// columns beyond it (look-ahead).
#include "factor.h"

#include <algorithm>

#include "common.h"
#include "gemm.h"
#include "solve.h"
#include "tsqr.h"

namespace miqr {

FactorWs carve_factor(double* base, const FactorLayout& L) {
  FactorWs w;
  int64_t off = 0;
  auto take = [&](int64_t n) {
    double* p = base ? base + off : nullptr;
    off += (n + 31) & ~int64_t(31);
    return p;
  };
  w.tsqr = take(L.tsqr);
  w.wa = take(L.wa);
  w.wb = take(L.wb);
  w.scratch = take(L.scratch);
  w.u1 = take(L.u1);
  w.u2 = take(L.u2);
  w.ua1 = take(L.ua1);
  w.ua2 = take(L.ua2);
  w.scratch_aux = take(L.scratch_aux);
  w.w_cap = L.wa;
  w.scratch_n = L.scratch;
  w.u_cap = L.u1;
  w.ua_cap = L.ua1;
  w.scratch_aux_n = L.scratch_aux;
  w.doubles = off;
  return w;
}

namespace {

struct EgCtx {
  hipStream_t s;
  double* A;
  int64_t lda;
  double* T;    // T of the problem being factored (FULL: whole; BLOCKED: the panel's block)
  int64_t t0;   // column of A where T's column 0 sits
  int64_t ldt;
  const Tuning* tune;
  const FactorWs* w;
  int update_compute;
  bool skip_spine_t;
  double* flops;
  hipError_t err = hipSuccess;
  // Thin Q and normalisation, emitted by a single TSQR panel itself.
  double* Q = nullptr;
  int64_t ldq = 0;
  int normalize = 0;
  double* sign = nullptr;
};

void run_gemm(EgCtx& e, const GemmDesc& d) {
  if (e.err != hipSuccess) return;
  e.err = gemm(d, e.s, e.w->scratch, e.w->scratch_n, e.flops);
}

double* t_at(EgCtx& e, int64_t r, int64_t c) {
  return e.T + (r - e.t0) + (c - e.t0) * e.ldt;
}

// Alg. 2 on the sub-problem with top-left corner (r0, c0), mk rows (to the
// bottom of A) and nk columns.  `spine`: the node lies on the right spine of
// the recursion (its T12 is never read by an update).
void eg(EgCtx& e, int64_t r0, int64_t c0, int64_t mk, int64_t nk, bool spine) {
  if (e.err != hipSuccess) return;
  double* A = e.A;
  const int64_t lda = e.lda, ldt = e.ldt;
  const Tuning& tu = *e.tune;
  const int64_t n1 = eg_split(nk, tu);
  if (n1 == 0) {
    // Base case: a TSQR panel (App. C) of width nk <= b*.
    int lr = tu.leaf_rows, ch = tu.chain, ar = tu.arity;
    if (lr == 0 || ch == 0 || ar == 0) {
      int a = 0, b = 0, c = 0;
      tsqr_auto(mk, (int)nk, &a, &b, &c);
      if (lr == 0) lr = a;
      if (ch == 0) ch = b;
      if (ar == 0) ar = c;
    }
    TsqrPlan p = tsqr_plan(mk, (int)nk, lr, ch, ar, e.w->tsqr);
    e.err = tsqr_factor(p, e.s, A + r0 + c0 * lda, lda, t_at(e, c0, c0), ldt, e.Q, e.ldq,
                        e.normalize, e.sign);
    return;
  }
  const int64_t n2 = nk - n1;
  if (n1 * n2 > e.w->w_cap) {
    // The layout is sized from every node; reaching this means the two
    // disagree, and running on would overwrite the neighbouring regions.
    e.err = hipErrorInvalidValue;
    return;
  }
  eg(e, r0, c0, mk, n1, false);
  double* VL = A + r0 + c0 * lda;
  double* C = A + r0 + (c0 + n1) * lda;
  double* TL = t_at(e, c0, c0);
  GemmDesc d;
  // M1 = V_L^T C
  d = GemmDesc();
  d.ta = 'T'; d.tb = 'N'; d.M = n1; d.N = n2; d.K = mk;
  d.A = VL; d.lda = lda; d.maskA = MASK_UNIT_LOWER;
  d.B = C; d.ldb = lda; d.C = e.w->wa; d.ldc = n1; d.compute = e.update_compute;
  run_gemm(e, d);
  // M2 = T_L^T M1
  d = GemmDesc();
  d.ta = 'T'; d.tb = 'N'; d.M = n1; d.N = n2; d.K = n1;
  d.A = TL; d.lda = ldt; d.maskA = MASK_UPPER;
  d.B = e.w->wa; d.ldb = n1; d.C = e.w->wb; d.ldc = n1;
  run_gemm(e, d);
  // [B12; B22] = C - V_L M2
  d = GemmDesc();
  d.ta = 'N'; d.tb = 'N'; d.M = mk; d.N = n2; d.K = n1; d.alpha = -1.0; d.beta = 1.0;
  d.A = VL; d.lda = lda; d.maskA = MASK_UNIT_LOWER;
  d.B = e.w->wb; d.ldb = n1; d.C = C; d.ldc = lda; d.compute = e.update_compute;
  run_gemm(e, d);
  eg(e, r0 + n1, c0 + n1, mk - n1, n2, spine);
  if (spine && e.skip_spine_t) return;
  double* VR = A + (r0 + n1) + (c0 + n1) * lda;
  double* TR = t_at(e, c0 + n1, c0 + n1);
  // M3 = V_L^T [0; V_R] = V_L[n1:, :]^T V_R
  d = GemmDesc();
  d.ta = 'T'; d.tb = 'N'; d.M = n1; d.N = n2; d.K = mk - n1;
  d.A = A + (r0 + n1) + c0 * lda; d.lda = lda;
  d.B = VR; d.ldb = lda; d.maskB = MASK_UNIT_LOWER; d.C = e.w->wa; d.ldc = n1;
  run_gemm(e, d);
  // M4 = M3 T_R
  d = GemmDesc();
  d.ta = 'N'; d.tb = 'N'; d.M = n1; d.N = n2; d.K = n2;
  d.A = e.w->wa; d.lda = n1; d.B = TR; d.ldb = ldt; d.maskB = MASK_UPPER;
  d.C = e.w->wb; d.ldc = n1;
  run_gemm(e, d);
  // T12 = -T_L M4
  d = GemmDesc();
  d.ta = 'N'; d.tb = 'N'; d.M = n1; d.N = n2; d.K = n1; d.alpha = -1.0;
  d.A = TL; d.lda = ldt; d.maskA = MASK_UPPER; d.B = e.w->wb; d.ldb = n1;
  d.C = t_at(e, c0, c0 + n1); d.ldc = ldt;
  run_gemm(e, d);
}

// C <- C - V (op(T) (V^T C)) for V (mk x w, unit lower, in A) and C
// (mk x ncols): the compact-WY update of Sec. 2.3.  op(T) = T^T applies Q^T
// (the factorisation's trailing update), op(T) = T applies Q.
hipError_t wy_update(hipStream_t s, int64_t mk, int64_t w, int64_t ncols, const double* V,
                     int64_t lda, const double* T, int64_t ldt, char top, double* C, int64_t ldc,
                     double* W1, double* W2, double* scratch, int64_t scratch_n, int compute,
                     double* flops) {
  if (ncols <= 0 || w <= 0) return hipSuccess;
  GemmDesc d;
  d.ta = 'T'; d.tb = 'N'; d.M = w; d.N = ncols; d.K = mk;
  d.A = V; d.lda = lda; d.maskA = MASK_UNIT_LOWER; d.B = C; d.ldb = ldc; d.C = W1; d.ldc = w;
  d.compute = compute;
  hipError_t e = gemm(d, s, scratch, scratch_n, flops);
  if (e != hipSuccess) return e;
  d = GemmDesc();
  d.ta = top; d.tb = 'N'; d.M = w; d.N = ncols; d.K = w;
  d.A = T; d.lda = ldt; d.maskA = MASK_UPPER; d.B = W1; d.ldb = w; d.C = W2; d.ldc = w;
  e = gemm(d, s, scratch, scratch_n, flops);
  if (e != hipSuccess) return e;
  d = GemmDesc();
  d.ta = 'N'; d.tb = 'N'; d.M = mk; d.N = ncols; d.K = w; d.alpha = -1.0; d.beta = 1.0;
  d.A = V; d.lda = lda; d.maskA = MASK_UNIT_LOWER; d.B = W2; d.ldb = w; d.C = C; d.ldc = ldc;
  d.compute = compute;
  return gemm(d, s, scratch, scratch_n, flops);
}

hipError_t factor_full(hipStream_t s, const Tuning& t, const FactorWs& w, const FactorArgs& a,
                       double* flops) {
  EgCtx e;
  e.s = s;
  e.A = a.A;
  e.lda = a.lda;
  e.T = a.T;
  e.t0 = 0;
  e.ldt = a.ldt;
  e.tune = &t;
  e.w = &w;
  e.update_compute = a.update_compute;
  e.skip_spine_t = a.skip_spine_t;
  e.flops = flops;
  const bool single = a.n <= t.bstar && a.m > a.n;
  if (single) {
    e.Q = a.Q;
    e.ldq = a.ldq;
    e.normalize = a.normalize;
    e.sign = a.sign;
  }
  eg(e, 0, 0, a.m, a.n, true);
  return e.err;
}

hipError_t factor_blocked(hipStream_t s, const Lookahead& la, const Tuning& t, const FactorWs& w,
                          const FactorArgs& a, double* flops) {
  const int64_t m = a.m, n = a.n, nb = std::min<int64_t>(std::max<int64_t>(t.nb, 1), n);
  double* A = a.A;
  const int64_t lda = a.lda;
  const bool single = n <= t.bstar && m > n;
  auto factor_panel = [&](int64_t j) -> hipError_t {
    const int64_t wd = std::min(nb, n - j);
    EgCtx e;
    e.s = s;
    e.A = A;
    e.lda = lda;
    e.T = a.T + j * a.ldt;
    e.t0 = j;
    e.ldt = a.ldt;
    e.tune = &t;
    e.w = &w;
    e.update_compute = a.update_compute;
    e.skip_spine_t = false;
    e.flops = flops;
    if (single) {
      e.Q = a.Q;
      e.ldq = a.ldq;
      e.normalize = a.normalize;
      e.sign = a.sign;
    }
    eg(e, j, j, m - j, wd, false);
    return e.err;
  };
  // Trailing update of panel j on columns [c1, c2).
  auto update = [&](hipStream_t st, int64_t j, int64_t c1, int64_t c2, double* W1, double* W2,
                    int64_t cap, double* sc, int64_t scn) -> hipError_t {
    const int64_t wd = std::min(nb, n - j), nc = c2 - c1;
    if (nc <= 0) return hipSuccess;
    if (wd * nc > cap) return hipErrorInvalidValue;
    return wy_update(st, m - j, wd, nc, A + j + j * lda, lda, a.T + j * a.ldt, a.ldt, 'T',
                     A + j + c1 * lda, lda, W1, W2, sc, scn, a.update_compute, flops);
  };
  constexpr int64_t kAuxChunk = 3072;  // columns per look-ahead update launch group
  const bool ahead = t.lookahead && la.aux && la.ev_panel && la.ev_update;
  hipError_t e = factor_panel(0);
  for (int64_t j = 0; j < n && e == hipSuccess; j += nb) {
    const int64_t wd = std::min(nb, n - j);
    const int64_t c1 = j + wd;                       // first column of panel k + 1
    if (c1 >= n) break;
    const int64_t c2 = std::min(n, c1 + nb);         // end of panel k + 1
    if (ahead && c2 < n) {
      // The columns beyond panel k + 1 go to the second stream once panel k
      // is factored; panel k + 1 is updated and factored here meanwhile.
      e = hipEventRecord(la.ev_panel, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(la.aux, la.ev_panel, 0);
      // In column chunks: a blocked TSQR workgroup needs a CU with no GEMM
      // workgroup on it, and the end of each chunk's launches drains CUs for
      // the panel kernels waiting on the main stream (3072 columns measured
      // best: 16384^2 alone 245 -> 233 ms; 2048 and 4096 in between, 1024
      // slower than no chunks).
      for (int64_t cc = c2; cc < n && e == hipSuccess; cc += kAuxChunk)
        e = update(la.aux, j, cc, std::min<int64_t>(n, cc + kAuxChunk), w.ua1, w.ua2, w.ua_cap,
                   w.scratch_aux, w.scratch_aux_n);
      if (e == hipSuccess) e = hipEventRecord(la.ev_update, la.aux);
      if (e == hipSuccess) e = update(s, j, c1, c2, w.u1, w.u2, w.u_cap, w.scratch, w.scratch_n);
      if (e == hipSuccess) e = factor_panel(c1);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, la.ev_update, 0);
    } else {
      if (ahead) {
        e = update(s, j, c1, n, w.u1, w.u2, w.u_cap, w.scratch, w.scratch_n);
      } else {
        // One stream: the whole trailing matrix at once (its temporaries are
        // the look-ahead stream's, sized for every column after the first
        // panel).
        e = update(s, j, c1, n, w.ua1, w.ua2, w.ua_cap, w.scratch_aux, w.scratch_aux_n);
      }
      if (e == hipSuccess) e = factor_panel(c1);
    }
  }
  return e;
}

}  // namespace

hipError_t run_factor(hipStream_t s, const Lookahead& la, const Tuning& t, const FactorWs& w,
                      const FactorArgs& a, double* flops) {
  const bool blocked = t.t_layout == T_BLOCKED;
  const int64_t nb = blocked ? std::min<int64_t>(std::max<int64_t>(t.nb, 1), a.n) : a.n;
  zero_block_lower(s, a.n, nb, a.T, a.ldt);
  hipError_t e = blocked ? factor_blocked(s, la, t, w, a, flops) : factor_full(s, t, w, a, flops);
  if (e != hipSuccess) return e;
  if (a.m == a.n) {
    const int64_t jl = blocked ? ((a.n - 1) / nb) * nb : 0;
    square_last_column(s, a.n, a.A, a.lda, a.T + (a.n - 1) * a.ldt, a.n - jl);
  }
  const bool single = a.n <= t.bstar && a.m > a.n;
  if (!single) {
    if (a.normalize) normalize_r(s, a.n, a.A, a.lda, a.sign);
    if (a.Q) {
      if (blocked) {
        e = form_q_blocked(s, a.m, a.n, a.A, a.lda, a.T, a.ldt, nb, a.normalize ? a.sign : nullptr,
                           a.Q, a.ldq, w.ua1, w.ua2, w.scratch_aux, w.scratch_aux_n);
      } else {
        // Q = [I; 0] - V (T V_top^T), V_top the unit lower n x n top of V.
        GemmDesc d;
        d.ta = 'N'; d.tb = 'T'; d.M = a.n; d.N = a.n; d.K = a.n;
        d.A = a.T; d.lda = a.ldt; d.maskA = MASK_UPPER; d.B = a.A; d.ldb = a.lda;
        d.maskB = MASK_UNIT_LOWER; d.C = w.ua1; d.ldc = a.n;
        e = gemm(d, s, w.scratch, w.scratch_n);
        if (e == hipSuccess) {
          d = GemmDesc();
          d.ta = 'N'; d.tb = 'N'; d.M = a.m; d.N = a.n; d.K = a.n; d.alpha = -1.0; d.beta = 0.0;
          d.add_identity = 1;
          d.A = a.A; d.lda = a.lda; d.maskA = MASK_UNIT_LOWER; d.B = w.ua1; d.ldb = a.n;
          d.C = a.Q; d.ldc = a.ldq;
          e = gemm(d, s, w.scratch, w.scratch_n);
        }
        if (e == hipSuccess && a.normalize) scale_columns(s, a.m, a.n, a.Q, a.ldq, a.sign);
      }
    }
  }
  if (e == hipSuccess) e = hipGetLastError();
  return e;
}

hipError_t apply_q_full(hipStream_t s, char trans, int64_t m, int64_t n, int64_t k,
                        const double* VR, int64_t lda, const double* T, int64_t ldt, double* C,
                        int64_t ldc, double* W1, double* W2, double* scratch, int64_t scratch_n) {
  if (k == 0) return hipSuccess;
  return wy_update(s, m, n, k, VR, lda, T, ldt, trans == 'T' ? 'T' : 'N', C, ldc, W1, W2, scratch,
                   scratch_n, COMPUTE_F64, nullptr);
}

hipError_t apply_q_blocked(hipStream_t s, char trans, int64_t m, int64_t n, int64_t k,
                           const double* VR, int64_t lda, const double* T, int64_t ldt, int64_t nb,
                           double* C, int64_t ldc, double* W1, double* W2, double* scratch,
                           int64_t scratch_n) {
  if (k == 0) return hipSuccess;
  nb = std::min<int64_t>(std::max<int64_t>(nb, 1), n);
  const int64_t K = (n + nb - 1) / nb;
  // Q = Q_0 Q_1 ... Q_{K-1}: Q^T C applies panel 0 first, Q C the last first.
  for (int64_t q = 0; q < K; ++q) {
    const int64_t p = trans == 'T' ? q : K - 1 - q;
    const int64_t j = p * nb, wd = std::min(nb, n - j);
    hipError_t e = wy_update(s, m - j, wd, k, VR + j + j * lda, lda, T + j * ldt, ldt,
                             trans == 'T' ? 'T' : 'N', C + j, ldc, W1, W2, scratch, scratch_n,
                             COMPUTE_F64, nullptr);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t apply_qt_spine(hipStream_t s, int64_t m, int64_t n, int64_t k, const double* VR,
                          int64_t lda, const double* T, int64_t ldt, double* C, int64_t ldc,
                          const Tuning& t, double* W1, double* W2, double* scratch,
                          int64_t scratch_n) {
  int64_t r0 = 0, c0 = 0, mk = m, nk = n;
  for (;;) {
    const int64_t n1 = eg_split(nk, t);
    const int64_t w = n1 == 0 ? nk : n1;
    hipError_t e = apply_q_full(s, 'T', mk, w, k, VR + r0 + c0 * lda, lda, T + c0 + c0 * ldt, ldt,
                                C + r0, ldc, W1, W2, scratch, scratch_n);
    if (e != hipSuccess || w == nk) return e;
    r0 += w;
    c0 += w;
    mk -= w;
    nk -= w;
  }
}

hipError_t form_q_blocked(hipStream_t s, int64_t m, int64_t n, const double* VR, int64_t lda,
                          const double* T, int64_t ldt, int64_t nb, const double* sign, double* Q,
                          int64_t ldq, double* W1, double* W2, double* scratch,
                          int64_t scratch_n) {
  nb = std::min<int64_t>(std::max<int64_t>(nb, 1), n);
  set_identity(s, m, n, Q, ldq);
  // Q [I; 0] = Q_0 (Q_1 (... Q_{K-1} [I; 0])): panel p touches rows >= j_p, and
  // the columns left of j_p are still unit vectors there, so only the block
  // Q[j_p:, j_p:] changes.
  const int64_t K = (n + nb - 1) / nb;
  for (int64_t p = K - 1; p >= 0; --p) {
    const int64_t j = p * nb, wd = std::min(nb, n - j);
    hipError_t e = wy_update(s, m - j, wd, n - j, VR + j + j * lda, lda, T + j * ldt, ldt, 'N',
                             Q + j + j * ldq, ldq, W1, W2, scratch, scratch_n, COMPUTE_F64,
                             nullptr);
    if (e != hipSuccess) return e;
  }
  if (sign) scale_columns(s, m, n, Q, ldq, sign);
  return hipGetLastError();
}

}  // namespace miqr

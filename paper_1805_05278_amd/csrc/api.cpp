// C ABI of libmiqr: handle and workspace management, the Elmroth-Gustavson
// recursion driver (Alg. 2), apply/form Q, triangular solve and least squares.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "batched.h"
#include "common.h"
#include "factor.h"
#include "gemm.h"
#include "handle.h"
#include "miqr.h"
#include "noalloc.h"
#include "plan.h"
#include "profiler.h"
#include "solve.h"
#include "tsqr.h"

using namespace miqr;



namespace {
// Points the launch-site timer at the handle for the duration of an entry
// point.  It also clears the thread's last-error state first: hipGetLastError
// reports the last failure of any runtime call on the thread, and the entry
// point's launch checks must not pick up an unrelated earlier one.
struct ProfScope {
  KernelTimer* prev;
  explicit ProfScope(miqr_handle h) : prev(g_timer) {
    (void)hipGetLastError();
    g_timer = (h && h->profiling) ? &h->timer : nullptr;
  }
  ~ProfScope() { g_timer = prev; }
};
}  // namespace

namespace {

miqr_status fail(miqr_handle h, miqr_status st, const std::string& msg) {
  if (h) h->err = msg;
  return st;
}

miqr_status hip_fail(miqr_handle h, hipError_t e, const char* where) {
  return fail(h, MIQR_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Drop every captured factorisation graph (their launches name workspace
// addresses that are about to change, or the handle is going away).
void clear_graphs(miqr_handle h) {
  for (auto& kv : h->graph_cache) hipGraphExecDestroy(kv.second.exec);
  h->graph_cache.clear();
}

miqr_status ensure_ws(miqr_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return MIQR_OK;
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return hip_fail(h, e, "hipSetDevice");
  if (h->ws) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(h, e, "hipDeviceSynchronize");
    clear_graphs(h);
    hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = std::max<size_t>(bytes, (size_t)64 << 20);
  e = hipMalloc((void**)&h->ws, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    h->ws = nullptr;
    return fail(h, MIQR_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
  }
  h->ws_bytes = want;
  return MIQR_OK;
}

// Bump allocator over the handle's workspace (doubles, 256-byte aligned).
struct Arena {
  double* base;
  int64_t off = 0;
  double* take(int64_t n) {
    double* p = base ? base + off : nullptr;
    off += (n + 31) & ~int64_t(31);
    return p;
  }
};

bool bad_ptr(const void* p) { return p == nullptr; }

// Captured factorisation graphs kept per handle (all dropped when full).
constexpr size_t kMaxGraphs = 64;

// Validation of the tuning and output options shared by the entry points
// (h may be null: the message is then dropped).
miqr_status check_opts(miqr_handle h, int64_t m, const qr_opts* o) {
  if (!o) return MIQR_OK;
  if (o->precision != MIQR_FP64 && o->precision != MIQR_MIXED_FP32 &&
      o->precision != MIQR_MIXED_BF16)
    return fail(h, MIQR_EINVAL, "bad precision");
  if (o->b < 0 || o->b > kMaxB)
    return fail(h, MIQR_EINVAL, "b must be in [0, " + std::to_string(kMaxB) + "]");
  if (o->bstar < 0 || o->bstar > kNB) return fail(h, MIQR_EINVAL, "bstar must be in [0, 64]");
  if (o->b > 0 && o->bstar > o->b) return fail(h, MIQR_EINVAL, "bstar must not exceed b");
  if (o->nb < 0 || o->nb > kMaxNB)
    return fail(h, MIQR_EINVAL, "nb must be in [0, " + std::to_string(kMaxNB) + "]");
  if (o->t_layout != MIQR_T_FULL && o->t_layout != MIQR_T_BLOCKED)
    return fail(h, MIQR_EINVAL, "bad t_layout");
  if (o->leaf_rows != 0 && o->leaf_rows != 128 && o->leaf_rows != 256)
    return fail(h, MIQR_EINVAL, "leaf_rows must be 0, 128 or 256");
  if (o->chain < 0 || o->arity < 0 || o->arity == 1)
    return fail(h, MIQR_EINVAL, "chain must be >= 0 and arity 0 or >= 2");
  if (o->normalize && !o->sign_out) return fail(h, MIQR_EINVAL, "normalize needs sign_out");
  if (o->Q && o->ldq < m) return fail(h, MIQR_EINVAL, "ldq < m");
  return MIQR_OK;
}

// The look-ahead stream and events of the handle (created on first use, at
// the default priority).
miqr_status ensure_lookahead(miqr_handle h, Lookahead* la) {
  hipError_t e = hipSuccess;
  if (!h->aux) e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
  if (e == hipSuccess && !h->ev_panel)
    e = hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming);
  if (e == hipSuccess && !h->ev_update)
    e = hipEventCreateWithFlags(&h->ev_update, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(h, e, "look-ahead stream");
  la->aux = h->aux;
  la->ev_panel = h->ev_panel;
  la->ev_update = h->ev_update;
  return MIQR_OK;
}

// Tuning for a call, through the handle's cache (the cost model's choice
// depends only on the shape and the fields the caller fixed).
Tuning tuning_for(miqr_handle h, int64_t m, int64_t n, const qr_opts* o, bool lstsq) {
  TuneKey k{m, n, lstsq ? 1 : 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (o) {
    k.b = o->b;
    k.bstar = o->bstar;
    k.nb = o->nb;
    k.leaf_rows = o->leaf_rows;
    k.chain = o->chain;
    k.arity = o->arity;
    k.layout = o->t_layout;
    k.nola = o->no_lookahead;
  }
  if (h) {
    auto it = h->tune_cache.find(k);
    if (it != h->tune_cache.end()) return it->second;
  }
  const Tuning t = choose_tuning(m, n, o, lstsq);
  if (h) {
    if (h->tune_cache.size() > 4096) h->tune_cache.clear();
    h->tune_cache[k] = t;
  }
  return t;
}

// Rows of T a factorisation writes: n (FULL) or the top-level panel width.
int64_t t_rows(const Tuning& t, int64_t n) {
  return t.t_layout == T_BLOCKED ? std::min<int64_t>(std::max<int64_t>(t.nb, 1), n) : n;
}

// Factor with the given tuning, the workspace regions carved from `base`
// (FactorLayout order).
miqr_status factor_with(miqr_handle h, hipStream_t s, const Tuning& tune, const FactorWs& w,
                        const FactorArgs& a) {
  Lookahead la;
  if (tune.t_layout == T_BLOCKED && tune.lookahead) {
    miqr_status st = ensure_lookahead(h, &la);
    if (st != MIQR_OK) return st;
  }
  double flops = 0.0;
  hipError_t e = run_factor(s, la, tune, w, a, &flops);
  if (e != hipSuccess) return hip_fail(h, e, "qr_factor");
  h->gemm_flops = flops;
  return MIQR_OK;
}

// The factorisation as one graph launch on s: the launch sequence of this
// key is captured once (on the handle's capture stream, whose work is only
// recorded, never run), instantiated and kept; later calls with the same key
// replay it.  The same kernels in the same order give bitwise the same
// results as the eager launches.
miqr_status factor_graph(miqr_handle h, hipStream_t s, const Tuning& tune, const FactorWs& w,
                         const FactorArgs& a, int prec) {
  GraphKey k{a.m, a.n, a.lda, a.ldt, a.Q ? a.ldq : 0, a.A, a.T, a.Q, a.sign, h->ws,
             a.normalize, prec, tune.b, tune.bstar, tune.nb, tune.leaf_rows, tune.chain,
             tune.arity, tune.t_layout, tune.lookahead};
  auto it = h->graph_cache.find(k);
  if (it == h->graph_cache.end()) {
    hipError_t e = hipSuccess;
    if (!h->cap) e = hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(h, e, "capture stream");
    if (tune.t_layout == T_BLOCKED && tune.lookahead) {
      Lookahead la;  // created before the capture starts
      miqr_status st = ensure_lookahead(h, &la);
      if (st != MIQR_OK) return st;
    }
    e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
    const miqr_status st = factor_with(h, h->cap, tune, w, a);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(h->cap, &g);
    if (st != MIQR_OK || e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      (void)hipGetLastError();
      return st != MIQR_OK ? st : hip_fail(h, e, "hipStreamEndCapture");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
    if (h->graph_cache.size() >= kMaxGraphs) {
      e = hipDeviceSynchronize();  // no dropped graph may still be running
      if (e != hipSuccess) {
        hipGraphExecDestroy(x);
        return hip_fail(h, e, "hipDeviceSynchronize");
      }
      clear_graphs(h);
    }
    it = h->graph_cache.emplace(k, GraphEntry{x, h->gemm_flops}).first;
  }
  const hipError_t e = hipGraphLaunch(it->second.exec, s);
  if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
  h->gemm_flops = it->second.gemm_flops;
  return MIQR_OK;
}

// Factor in the handle's workspace (grown to the layout first); through a
// captured graph when the handle has graphs on (and per-kernel timing off:
// its events and host reads cannot be captured).
miqr_status do_factor(miqr_handle h, hipStream_t s, const Tuning& tune, const FactorArgs& a,
                      int prec = MIQR_FP64) {
  const FactorLayout L = factor_layout(a.m, a.n, tune, a.Q != nullptr);
  miqr_status st = ensure_ws(h, (size_t)L.total * sizeof(double));
  if (st != MIQR_OK) return st;
  const FactorWs w = carve_factor((double*)h->ws, L);
  if (h->graphs && !h->profiling) return factor_graph(h, s, tune, w, a, prec);
  return factor_with(h, s, tune, w, a);
}

// beta from the norms fa = ||A||_F, un = ||A^T r||, xn = ||x||, rn = ||r||,
// with the quotients taken before any product, so that no product of norms
// overflows: (un / fa / fa) / (xn + rn / fa).  NaN when a norm is not finite
// (a sum of squares overflowed: the estimate cannot decide, and callers treat
// it as not converged); 0 for x = 0 and r = 0.
double backward_from_norms(double fa, double un, double xn, double rn) {
  if (!(std::isfinite(fa) && std::isfinite(un) && std::isfinite(xn) && std::isfinite(rn)))
    return NAN;
  if (fa == 0.0) return un == 0.0 ? 0.0 : NAN;
  const double den = xn + rn / fa;
  return den > 0.0 ? (un / fa / fa) / den : 0.0;
}
// The larger of two estimates; a NaN one wins (std::max would drop it).
double worse_of(double w, double be) { return (be > w || be != be) ? be : w; }

// beta(x)_c = ||A^T r_c|| / (||A||_F (||A||_F ||x_c|| + ||r_c||)),
// r = b - A x, all FP64 on the device (A0, B0 originals; X solutions).  Rr
// (m x k) and U (n x k) are scratch, nrm 3k + n doubles.  Writes every
// right-hand side's value to out (host, k doubles) when given and returns the
// largest.  Synchronises the stream.
double backward_error_dev(hipStream_t s, int64_t m, int64_t n, int64_t k, const double* A0,
                          int64_t lda, const double* B0, int64_t ldb, const double* X,
                          int64_t ldx, double* Rr, double* U, double* nrm, double* sc, int64_t scn,
                          hipError_t* err, double* out = nullptr) {
  copy_matrix(s, m, k, B0, ldb, Rr, m);
  GemmDesc d;
  d.ta = 'N'; d.tb = 'N'; d.M = m; d.N = k; d.K = n; d.alpha = -1.0; d.beta = 1.0;
  d.A = A0; d.lda = lda; d.B = X; d.ldb = ldx; d.C = Rr; d.ldc = m;
  hipError_t e = gemm(d, s, sc, scn);
  d = GemmDesc();
  d.ta = 'T'; d.tb = 'N'; d.M = n; d.N = k; d.K = m;
  d.A = A0; d.lda = lda; d.B = Rr; d.ldb = m; d.C = U; d.ldc = n;
  if (e == hipSuccess) e = gemm(d, s, sc, scn);
  column_sumsq(s, m, k, Rr, m, nrm);
  column_sumsq(s, n, k, U, n, nrm + k);
  column_sumsq(s, n, k, X, ldx, nrm + 2 * k);
  column_sumsq(s, m, n, A0, lda, nrm + 3 * k);
  std::vector<double> hn(3 * k + n);
  if (e == hipSuccess)
    e = hipMemcpyAsync(hn.data(), nrm, sizeof(double) * hn.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  *err = e;
  if (e != hipSuccess) return 0.0;
  double fa = 0.0;
  for (int64_t j = 0; j < n; ++j) fa += hn[3 * k + j];
  fa = std::sqrt(fa);
  double worst = 0.0;
  for (int64_t c = 0; c < k; ++c) {
    const double rn = std::sqrt(hn[c]), gn = std::sqrt(hn[k + c]), xn = std::sqrt(hn[2 * k + c]);
    const double be = backward_from_norms(fa, gn, xn, rn);
    if (out) out[c] = be;
    worst = worse_of(worst, be);
  }
  return worst;
}

// Q^T B with the factors in the tuning's T layout (FULL factors from least
// squares have their right-spine T12 blocks unassembled).  W1, W2: n x k.
hipError_t apply_qt(hipStream_t s, const Tuning& t, int64_t m, int64_t n, int64_t k,
                    const double* A, int64_t lda, const double* T, int64_t ldt, double* B,
                    int64_t ldb, double* W1, double* W2, double* sc, int64_t scn) {
  if (t.t_layout == T_BLOCKED)
    return apply_q_blocked(s, 'T', m, n, k, A, lda, T, ldt, t.nb, B, ldb, W1, W2, sc, scn);
  return apply_qt_spine(s, m, n, k, A, lda, T, ldt, B, ldb, t, W1, W2, sc, scn);
}

// FP64 least squares on carved regions: factor, B <- Q^T B, singularity
// check, back substitution R x = (Q^T b)[0:n].
miqr_status lstsq_core(miqr_handle h, hipStream_t s, const Tuning& tune, const FactorWs& f,
                       int64_t m, int64_t n, int64_t k, double* A, int64_t lda, double* B,
                       int64_t ldb, double* T, double* W1, double* W2, qr_info* info) {
  FactorArgs a;
  a.m = m;
  a.n = n;
  a.A = A;
  a.lda = lda;
  a.T = T;
  a.ldt = t_rows(tune, n);
  a.update_compute = COMPUTE_F64;
  a.skip_spine_t = true;
  miqr_status st = factor_with(h, s, tune, f, a);
  if (st != MIQR_OK) return st;
  hipError_t e = apply_qt(s, tune, m, n, k, A, lda, T, a.ldt, B, ldb, W1, W2, f.scratch,
                          f.scratch_n);
  if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq apply");
  find_zero_diagonal(s, n, A, lda, h->dflag);
  int flag = 0;
  e = hipMemcpyAsync(&flag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq");
  if (flag) {
    if (info) info->singular_index = flag;
    return fail(h, MIQR_ESINGULAR, "R(" + std::to_string(flag - 1) + ") == 0");
  }
  e = solve_upper(s, n, k, A, lda, B, ldb, f.scratch, f.scratch_n);
  if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq solve");
  if (info) info->precision_used = MIQR_FP64;
  return MIQR_OK;
}

// Least squares with the mixed form: the factorisation runs with FP32/BF16
// trailing updates; the solution is refined in FP64 by conjugate gradients on
// min ||b - A R^{-1} y|| (CGLS, right preconditioner R, x = R^{-1} y), with
// every residual taken against the FP64 original of A.  It refines until the
// backward error beta(x) (worst right-hand side) is at most tol and has
// stopped improving (below 4u, or less than halved by the last iteration), so
// the result carries FP64 accuracy rather than just meeting the gate; it
// fails over to the FP64 path if the gate is not met within maxit steps, or
// as soon as the observed contraction rate shows it will not be.
struct MixedWs {
  double *T, *A0, *B0, *Rinv, *X, *Rr, *S, *P, *Tv, *Qv, *U, *W1, *W2, *nrm, *coef;
};

miqr_status lstsq_mixed(miqr_handle h, hipStream_t s, int64_t m, int64_t n, int64_t k, double* A,
                        int64_t lda, double* B, int64_t ldb, const qr_opts* o, int comp,
                        qr_info* info) {
  const Tuning tune = tuning_for(h, m, n, o, true);
  const FactorLayout L = factor_layout(m, n, tune);
  const int64_t tr = t_rows(tune, n);
  MixedWs w;
  FactorWs f;
  // The workspace size is taken from the same carving that assigns the
  // pointers (a dry run over a null base), so the two cannot disagree.
  auto carve = [&](double* base) {
    f = carve_factor(base, L);
    Arena ar{base};
    ar.off = f.doubles;
    w.T = ar.take(tr * n);
    w.Rinv = ar.take(n * n);
    w.A0 = ar.take(m * n);
    w.B0 = ar.take(m * k);
    w.Rr = ar.take(m * k);
    w.Qv = ar.take(m * k);
    w.X = ar.take(n * k);
    w.S = ar.take(n * k);
    w.P = ar.take(n * k);
    w.Tv = ar.take(n * k);
    w.U = ar.take(n * k);
    w.W1 = ar.take(n * k);
    w.W2 = ar.take(n * k);
    w.nrm = ar.take(4 * k + n + 8);
    w.coef = ar.take(2 * k + 8);
    return ar.off;
  };
  const int64_t need = carve(nullptr);
  miqr_status st = ensure_ws(h, (size_t)need * sizeof(double));
  if (st != MIQR_OK) return st;
  carve((double*)h->ws);
  const double tol = 1e-13, floor = 4.0 * 0x1p-53;
  const int maxit = 100;
  copy_matrix(s, m, n, A, lda, w.A0, m);
  copy_matrix(s, m, k, B, ldb, w.B0, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "lstsq_mixed copies");
  {
    FactorArgs a;
    a.m = m;
    a.n = n;
    a.A = A;
    a.lda = lda;
    a.T = w.T;
    a.ldt = tr;
    a.update_compute = comp;
    a.skip_spine_t = true;
    st = factor_with(h, s, tune, f, a);
    if (st != MIQR_OK) return st;
  }
  find_zero_diagonal(s, n, A, lda, h->dflag);
  int flag = 0;
  e = hipMemcpyAsync(&flag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(h, e, "lstsq_mixed singularity check");
  bool converged = false;
  int iters = 0;
  double worst = 0.0;
  auto G = [&](char ta, int64_t M, int64_t N, int64_t K, double alpha, const double* Ap,
               int64_t la, int ma, const double* Bp, int64_t lb, double beta, double* Cp,
               int64_t lc) {
    if (e != hipSuccess) return;
    GemmDesc d;
    d.ta = ta; d.tb = 'N'; d.M = M; d.N = N; d.K = K; d.alpha = alpha; d.beta = beta;
    d.A = Ap; d.lda = la; d.maskA = ma; d.B = Bp; d.ldb = lb; d.C = Cp; d.ldc = lc;
    e = gemm(d, s, f.scratch, f.scratch_n);
  };
  std::vector<double> hn(4 * k + n + 8), hc(2 * k + 8);
  auto fetch_norms = [&](int cnt) {
    if (e == hipSuccess)
      e = hipMemcpyAsync(hn.data(), w.nrm, sizeof(double) * cnt, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  };
  if (!flag) {
    // R^{-1} (upper): solve R Z = I.
    set_identity(s, n, n, w.Rinv, n);
    e = solve_upper(s, n, n, A, lda, w.Rinv, n, f.scratch, f.scratch_n);
    // x0 = R^{-1} (Q^T b)[0:n]
    copy_matrix(s, m, k, w.B0, m, w.Rr, m);
    if (e == hipSuccess)
      e = apply_qt(s, tune, m, n, k, A, lda, w.T, tr, w.Rr, m, w.W1, w.W2, f.scratch,
                   f.scratch_n);
    G('N', n, k, n, 1.0, w.Rinv, n, MASK_UPPER, w.Rr, m, 0.0, w.X, n);
    // ||A||_F
    column_sumsq(s, m, n, w.A0, m, w.nrm + 4 * k);
    fetch_norms(4 * k + n);
    double fa = 0.0;
    for (int64_t j = 0; j < n; ++j) fa += hn[4 * k + j];
    fa = std::sqrt(fa);
    // r = b - A x, u = A^T r, s = R^{-T} u, p = s
    copy_matrix(s, m, k, w.B0, m, w.Rr, m);
    G('N', m, k, n, -1.0, w.A0, m, MASK_NONE, w.X, n, 1.0, w.Rr, m);
    G('T', n, k, m, 1.0, w.A0, m, MASK_NONE, w.Rr, m, 0.0, w.U, n);
    G('T', n, k, n, 1.0, w.Rinv, n, MASK_UPPER, w.U, n, 0.0, w.S, n);
    copy_matrix(s, n, k, w.S, n, w.P, n);
    column_sumsq(s, n, k, w.S, n, w.nrm);
    column_sumsq(s, n, k, w.U, n, w.nrm + k);
    column_sumsq(s, n, k, w.X, n, w.nrm + 2 * k);
    column_sumsq(s, m, k, w.Rr, m, w.nrm + 3 * k);
    fetch_norms(4 * k);
    std::vector<double> gam(k);
    auto backward = [&]() {
      worst = 0.0;
      for (int64_t c = 0; c < k; ++c) {
        const double un = std::sqrt(hn[k + c]), xn = std::sqrt(hn[2 * k + c]),
                     rn = std::sqrt(hn[3 * k + c]);
        worst = worse_of(worst, backward_from_norms(fa, un, xn, rn));
      }
    };
    for (int64_t c = 0; c < k; ++c) gam[c] = hn[c];
    backward();
    double prev = worst;
    std::vector<double> hist{worst};
    auto settled = [&]() { return worst <= tol && (worst <= floor || worst > 0.5 * prev); };
    bool done = worst <= floor;
    // A NaN estimate (overflowing norms) cannot improve: fall back at once.
    while (!done && worst == worst && iters < maxit && e == hipSuccess) {
      ++iters;
      // t = R^{-1} p, q = A t, alpha = gamma / ||q||^2
      G('N', n, k, n, 1.0, w.Rinv, n, MASK_UPPER, w.P, n, 0.0, w.Tv, n);
      G('N', m, k, n, 1.0, w.A0, m, MASK_NONE, w.Tv, n, 0.0, w.Qv, m);
      column_sumsq(s, m, k, w.Qv, m, w.nrm);
      fetch_norms(k);
      bool stop = false;
      for (int64_t c = 0; c < k; ++c) {
        hc[c] = (hn[c] > 0.0) ? gam[c] / hn[c] : 0.0;
        if (hn[c] == 0.0) stop = true;
      }
      if (stop) break;
      if (e == hipSuccess)
        e = hipMemcpyAsync(w.coef, hc.data(), sizeof(double) * k, hipMemcpyHostToDevice, s);
      axpy_cols(s, n, k, 1.0, w.coef, w.Tv, n, w.X, n);
      axpy_cols(s, m, k, -1.0, w.coef, w.Qv, m, w.Rr, m);
      // u = A^T r, backward error, s = R^{-T} u, p = s + beta p
      G('T', n, k, m, 1.0, w.A0, m, MASK_NONE, w.Rr, m, 0.0, w.U, n);
      G('T', n, k, n, 1.0, w.Rinv, n, MASK_UPPER, w.U, n, 0.0, w.S, n);
      column_sumsq(s, n, k, w.S, n, w.nrm);
      column_sumsq(s, n, k, w.U, n, w.nrm + k);
      column_sumsq(s, n, k, w.X, n, w.nrm + 2 * k);
      column_sumsq(s, m, k, w.Rr, m, w.nrm + 3 * k);
      fetch_norms(4 * k);
      prev = worst;
      backward();
      if (settled() || worst != worst) break;
      // Give up early (and fall back) when the contraction over the last five
      // iterations cannot reach the gate within the iteration cap.
      hist.push_back(worst);
      if (hist.size() >= 8) {
        const double rate = std::pow(worst / hist[hist.size() - 6], 0.2);
        if (!(rate < 1.0) || worst * std::pow(rate, maxit - iters) > tol) break;
      }
      for (int64_t c = 0; c < k; ++c) {
        hc[k + c] = (gam[c] > 0.0) ? hn[c] / gam[c] : 0.0;
        gam[c] = hn[c];
      }
      if (e == hipSuccess)
        e = hipMemcpyAsync(w.coef + k, hc.data() + k, sizeof(double) * k, hipMemcpyHostToDevice, s);
      xpby_cols(s, n, k, w.S, n, w.coef + k, w.P, n);
    }
  }
  if (e != hipSuccess) return hip_fail(h, e, "lstsq_mixed refinement");
  converged = !flag && worst <= tol;
  if (converged) {
    copy_matrix(s, n, k, w.X, n, B, ldb);
    if (info) {
      info->iterations = iters;
      info->fallback = 0;
      info->precision_used = o ? o->precision : MIQR_FP64;
      info->backward_error = worst;
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "lstsq_mixed result");
    return MIQR_OK;
  }
  // Fallback: refactor the original in FP64.
  copy_matrix(s, m, n, w.A0, m, A, lda);
  copy_matrix(s, m, k, w.B0, m, B, ldb);
  st = lstsq_core(h, s, tune, f, m, n, k, A, lda, B, ldb, w.T, w.W1, w.W2, info);
  if (info) {
    info->iterations = iters;
    info->fallback = 1;
  }
  if (st != MIQR_OK) return st;
  if (info) {
    info->backward_error = backward_error_dev(s, m, n, k, w.A0, m, w.B0, m, B, ldb, w.Rr, w.U,
                                              w.nrm, f.scratch, f.scratch_n, &e);
    if (e != hipSuccess) return hip_fail(h, e, "lstsq_mixed fallback");
  }
  return fail(h, MIQR_ENOCONV, "refinement did not reach 1e-13; FP64 result returned");
}

// Pinned host staging for `count` tasks and 2 `count` ints (statuses, then
// refinement iterations).  Waits for the previous
// upload out of the staging buffer before it may be rewritten.
miqr_status ensure_pinned(miqr_handle h, int64_t count) {
  hipError_t e = hipSuccess;
  if (!h->table_ev) {
    e = hipEventCreateWithFlags(&h->table_ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(h, e, "hipEventCreate");
  } else {
    e = hipEventSynchronize(h->table_ev);
    if (e != hipSuccess) return hip_fail(h, e, "hipEventSynchronize");
  }
  if (count <= h->pin_cap) return MIQR_OK;
  if (h->pin_tasks) hipHostFree(h->pin_tasks);
  if (h->pin_status) hipHostFree(h->pin_status);
  h->pin_tasks = nullptr;
  h->pin_status = nullptr;
  h->pin_cap = 0;
  const int64_t cap = std::max<int64_t>(count, 1024);
  e = hipHostMalloc((void**)&h->pin_tasks, batch_table_bytes(cap), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void**)&h->pin_status, 2 * cap * sizeof(int32_t), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, MIQR_ENOMEM, "pinned staging allocation failed");
  }
  h->pin_cap = cap;
  return MIQR_OK;
}

// Algorithmic bytes and flops of one batched problem (read [A | B], write R
// into A and X into B; Householder QR of A plus Q^T B and back substitution).
void batch_item_cost(const qr_batch_item& it, double* bytes, double* flops) {
  const double m = (double)it.m, n = (double)it.n, k = (double)it.nrhs;
  *bytes += 8.0 * (m * (n + k) + n * (n + 1) / 2 + n * k);
  *flops += 2.0 * m * n * n - 2.0 * n * n * n / 3.0 + 4.0 * m * n * k + n * n * k;
}

}  // namespace

extern "C" {

miqr_status miqr_create(miqr_handle* handle, int device) {
  if (!handle) return MIQR_EINVAL;
  *handle = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) {
    (void)hipGetLastError();
    return MIQR_EHIP;
  }
  if (device < 0 || device >= count) return MIQR_EINVAL;
  miqr_ctx* c = new miqr_ctx();
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || hipMalloc((void**)&c->dflag, 256) != hipSuccess) {
    delete c;
    return MIQR_EHIP;
  }
  // The static workspace of qr_factor_noalloc on this device.
  if (noalloc_setup(device) != hipSuccess) {
    hipFree(c->dflag);
    delete c;
    return MIQR_EHIP;
  }
  *handle = c;
  return MIQR_OK;
}

miqr_status miqr_destroy(miqr_handle h) {
  if (!h) return MIQR_EINVAL;
  hipSetDevice(h->device);
  hipDeviceSynchronize();
  clear_graphs(h);
  if (h->cap) hipStreamDestroy(h->cap);
  if (h->ws) hipFree(h->ws);
  if (h->dflag) hipFree(h->dflag);
  if (h->pin_tasks) hipHostFree(h->pin_tasks);
  if (h->pin_status) hipHostFree(h->pin_status);
  if (h->table_ev) hipEventDestroy(h->table_ev);
  if (h->ev_panel) hipEventDestroy(h->ev_panel);
  if (h->ev_update) hipEventDestroy(h->ev_update);
  if (h->aux) hipStreamDestroy(h->aux);
  delete h;
  return MIQR_OK;
}

const char* miqr_status_string(miqr_status s) {
  switch (s) {
    case MIQR_OK: return "success";
    case MIQR_EINVAL: return "invalid argument";
    case MIQR_ENOMEM: return "out of device memory";
    case MIQR_EHIP: return "HIP runtime error";
    case MIQR_ESINGULAR: return "R has an exactly zero diagonal entry";
    case MIQR_ENOCONV: return "iterative refinement did not converge (FP64 fallback used)";
    case MIQR_EBUSY: return "busy (no slot or memory available)";
    case MIQR_ENOTSUP: return "option combination not supported";
  }
  return "unknown status";
}

const char* miqr_last_error(miqr_handle h) { return h ? h->err.c_str() : ""; }

int64_t qr_workspace_size(int64_t m, int64_t n, const qr_opts* o) {
  if (m < n || n < 1) return 0;
  if (check_opts(nullptr, m, o) != MIQR_OK) return 0;
  const Tuning t = choose_tuning(m, n, o);
  return factor_layout(m, n, t, o && o->Q).total * (int64_t)sizeof(double);
}

int64_t qr_t_rows(int64_t m, int64_t n, const qr_opts* o) {
  if (m < n || n < 1) return 0;
  if (check_opts(nullptr, m, o) != MIQR_OK) return 0;
  return t_rows(choose_tuning(m, n, o), n);
}

int64_t qr_plan(int64_t m, int64_t n, const qr_opts* o, int lstsq, char* buf, int64_t len) {
  if (m < n || n < 1) return -1;
  if (check_opts(nullptr, m, o) != MIQR_OK) return -1;
  const std::string d = describe_plan(m, n, choose_tuning(m, n, o, lstsq != 0));
  if (buf && len > 0) {
    const size_t c = std::min<size_t>(d.size(), (size_t)len - 1);
    std::memcpy(buf, d.data(), c);
    buf[c] = 0;
  }
  return (int64_t)d.size();
}

double miqr_last_gemm_flops(miqr_handle h) { return h ? h->gemm_flops : 0.0; }

miqr_status miqr_profile_enable(miqr_handle h, int enable) {
  if (!h) return MIQR_EINVAL;
  if (enable) h->timer.clear();
  h->profiling = enable != 0;
  return MIQR_OK;
}

miqr_status miqr_graphs_enable(miqr_handle h, int enable) {
  if (!h) return MIQR_EINVAL;
  if (!enable && !h->graph_cache.empty()) {
    hipSetDevice(h->device);
    hipDeviceSynchronize();
    clear_graphs(h);
  }
  h->graphs = enable != 0;
  return MIQR_OK;
}

int64_t miqr_graph_count(miqr_handle h) { return h ? (int64_t)h->graph_cache.size() : 0; }

int miqr_profile_kernels(miqr_handle h) {
  if (!h) return 0;
  h->timer.collect();
  h->prof_names.clear();
  for (auto& kv : h->timer.totals) h->prof_names.push_back(kv.first);
  return (int)h->prof_names.size();
}

miqr_status miqr_profile_get(miqr_handle h, int index, char* name, int name_len, double* ms,
                             int64_t* launches, double* bytes, double* flops) {
  if (!h || index < 0 || index >= (int)h->prof_names.size()) return MIQR_EINVAL;
  const std::string& k = h->prof_names[index];
  const KernelTotals& t = h->timer.totals[k];
  if (name && name_len > 0) {
    std::strncpy(name, k.c_str(), (size_t)name_len - 1);
    name[name_len - 1] = 0;
  }
  if (ms) *ms = t.ms;
  if (launches) *launches = t.launches;
  if (bytes) *bytes = t.bytes;
  if (flops) *flops = t.flops;
  return MIQR_OK;
}

miqr_status qr_factor(miqr_handle h, void* stream, int64_t m, int64_t n, double* A, int64_t lda,
                      double* T, int64_t ldt, const qr_opts* o) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (n < 1 || m < n) return fail(h, MIQR_EINVAL, "need m >= n >= 1");
  if (lda < m) return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(A) || bad_ptr(T)) return fail(h, MIQR_EINVAL, "null matrix pointer");
  miqr_status st = check_opts(h, m, o);
  if (st != MIQR_OK) return st;
  const Tuning tune = tuning_for(h, m, n, o, false);
  if (ldt < t_rows(tune, n))
    return fail(h, MIQR_EINVAL, "ldt < " + std::to_string(t_rows(tune, n)) + " (rows of T)");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  const int prec = o ? o->precision : MIQR_FP64;
  FactorArgs a;
  a.m = m;
  a.n = n;
  a.A = A;
  a.lda = lda;
  a.T = T;
  a.ldt = ldt;
  a.update_compute = prec == MIQR_MIXED_FP32 ? COMPUTE_F32
                     : prec == MIQR_MIXED_BF16 ? COMPUTE_BF16 : COMPUTE_F64;
  if (o) {
    a.Q = o->Q;
    a.ldq = o->ldq;
    a.normalize = o->normalize;
    a.sign = o->sign_out;
  }
  return do_factor(h, (hipStream_t)stream, tune, a, prec);
}

miqr_status qr_factor_noalloc(miqr_handle h, void* stream, int64_t m, int64_t n, double* A,
                              int64_t lda, double* T, int64_t ldt, const qr_opts* o) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (n < 1 || m < n) return fail(h, MIQR_EINVAL, "need m >= n >= 1");
  if (lda < m) return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(A) || bad_ptr(T)) return fail(h, MIQR_EINVAL, "null matrix pointer");
  miqr_status st = check_opts(h, m, o);
  if (st != MIQR_OK) return st;
  // Every step on the caller's stream (no look-ahead stream or events).
  qr_opts one = o ? *o : qr_opts{};
  one.no_lookahead = 1;
  const Tuning tune = tuning_for(h, m, n, &one, false);
  if (ldt < t_rows(tune, n))
    return fail(h, MIQR_EINVAL, "ldt < " + std::to_string(t_rows(tune, n)) + " (rows of T)");
  double* base = noalloc_scratch(h->device);
  if (!base) return fail(h, MIQR_EHIP, "static workspace not set up on this device");
  // The regions of the factorisation, with the split-K partials given what
  // is left of the static array (the products split K only as far as their
  // partials fit, down to no split at all).
  FactorLayout L = factor_layout(m, n, tune, one.Q != nullptr);
  L.total -= ((L.scratch + 31) & ~int64_t(31)) + ((L.scratch_aux + 31) & ~int64_t(31));
  const int64_t spare = kNoallocDoubles - L.total;
  if (spare < 2 * 4096)
    return fail(h, MIQR_EINVAL,
                "workspace of " + std::to_string((L.total + 2 * 4096) * 8) +
                    " bytes exceeds the static " + std::to_string(kNoallocDoubles * 8) +
                    "-byte workspace of qr_factor_noalloc");
  L.scratch = ((spare / 2) & ~int64_t(31)) - 32;
  L.scratch_aux = L.scratch;
  L.total += 2 * (L.scratch + 32);
  const FactorWs w = carve_factor(base, L);
  if (w.doubles > kNoallocDoubles) return fail(h, MIQR_EINVAL, "static workspace too small");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  const int prec = one.precision;
  FactorArgs a;
  a.m = m;
  a.n = n;
  a.A = A;
  a.lda = lda;
  a.T = T;
  a.ldt = ldt;
  a.update_compute = prec == MIQR_MIXED_FP32 ? COMPUTE_F32
                     : prec == MIQR_MIXED_BF16 ? COMPUTE_BF16 : COMPUTE_F64;
  a.Q = one.Q;
  a.ldq = one.ldq;
  a.normalize = one.normalize;
  a.sign = one.sign_out;
  return factor_with(h, (hipStream_t)stream, tune, w, a);
}

miqr_status qr_apply_q(miqr_handle h, void* stream, char trans, int64_t m, int64_t n, int64_t k,
                       const double* VR, int64_t lda, const double* T, int64_t ldt, double* C,
                       int64_t ldc) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (trans != 'N' && trans != 'T') return fail(h, MIQR_EINVAL, "trans must be 'N' or 'T'");
  if (n < 1 || m < n || k < 0) return fail(h, MIQR_EINVAL, "need m >= n >= 1, k >= 0");
  if (lda < m || ldt < n || ldc < m) return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(VR) || bad_ptr(T) || bad_ptr(C)) return fail(h, MIQR_EINVAL, "null pointer");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  const int64_t scratch_n = std::max<int64_t>(int64_t(4) << 20, 4 * n * k);
  miqr_status st = ensure_ws(h, (size_t)(2 * n * k + scratch_n + 128) * sizeof(double));
  if (st != MIQR_OK) return st;
  Arena ar{(double*)h->ws};
  double* W1 = ar.take(n * k);
  double* W2 = ar.take(n * k);
  double* sc = ar.take(scratch_n);
  hipError_t e = apply_q_full((hipStream_t)stream, trans, m, n, k, VR, lda, T, ldt, C, ldc, W1, W2,
                              sc, scratch_n);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "qr_apply_q");
  return MIQR_OK;
}

miqr_status qr_apply_q_blocked(miqr_handle h, void* stream, char trans, int64_t m, int64_t n,
                               int64_t k, const double* VR, int64_t lda, const double* T,
                               int64_t ldt, int64_t nb, double* C, int64_t ldc) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (trans != 'N' && trans != 'T') return fail(h, MIQR_EINVAL, "trans must be 'N' or 'T'");
  if (n < 1 || m < n || k < 0 || nb < 1) return fail(h, MIQR_EINVAL, "need m >= n >= 1, k >= 0, nb >= 1");
  if (lda < m || ldt < std::min(nb, n) || ldc < m)
    return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(VR) || bad_ptr(T) || bad_ptr(C)) return fail(h, MIQR_EINVAL, "null pointer");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  const int64_t w = std::min(nb, n);
  const int64_t scratch_n = std::max<int64_t>(int64_t(4) << 20, 4 * w * k);
  miqr_status st = ensure_ws(h, (size_t)(2 * w * k + scratch_n + 128) * sizeof(double));
  if (st != MIQR_OK) return st;
  Arena ar{(double*)h->ws};
  double* W1 = ar.take(w * k);
  double* W2 = ar.take(w * k);
  double* sc = ar.take(scratch_n);
  hipError_t e = apply_q_blocked((hipStream_t)stream, trans, m, n, k, VR, lda, T, ldt, nb, C, ldc,
                                 W1, W2, sc, scratch_n);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "qr_apply_q_blocked");
  return MIQR_OK;
}

miqr_status qr_form_q(miqr_handle h, void* stream, int64_t m, int64_t n, const double* VR,
                      int64_t lda, const double* T, int64_t ldt, const double* sign, double* Q,
                      int64_t ldq) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (n < 1 || m < n) return fail(h, MIQR_EINVAL, "need m >= n >= 1");
  if (lda < m || ldt < n || ldq < m) return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(VR) || bad_ptr(T) || bad_ptr(Q)) return fail(h, MIQR_EINVAL, "null pointer");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  // Q = [I; 0] - V (T V_top^T), V_top the unit lower n x n top of V.
  const int64_t scratch_n = std::max<int64_t>(int64_t(4) << 20, 2 * n * n);
  miqr_status st = ensure_ws(h, (size_t)(n * n + scratch_n + 64) * sizeof(double));
  if (st != MIQR_OK) return st;
  Arena ar{(double*)h->ws};
  double* W = ar.take(n * n);
  double* sc = ar.take(scratch_n);
  GemmDesc d;
  d.ta = 'N'; d.tb = 'T'; d.M = n; d.N = n; d.K = n;
  d.A = T; d.lda = ldt; d.maskA = MASK_UPPER; d.B = VR; d.ldb = lda; d.maskB = MASK_UNIT_LOWER;
  d.C = W; d.ldc = n;
  hipError_t e = gemm(d, s, sc, scratch_n);
  if (e == hipSuccess) {
    // Q = [I; 0] - V W in one pass (the identity is added in the epilogue).
    d = GemmDesc();
    d.ta = 'N'; d.tb = 'N'; d.M = m; d.N = n; d.K = n; d.alpha = -1.0; d.beta = 0.0;
    d.add_identity = 1;
    d.A = VR; d.lda = lda; d.maskA = MASK_UNIT_LOWER; d.B = W; d.ldb = n; d.C = Q; d.ldc = ldq;
    e = gemm(d, s, sc, scratch_n);
  }
  if (e == hipSuccess && sign) scale_columns(s, m, n, Q, ldq, sign);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(h, e, "qr_form_q");
  return MIQR_OK;
}

miqr_status qr_solve_r(miqr_handle h, void* stream, int64_t n, int64_t nrhs, const double* VR,
                       int64_t lda, double* X, int64_t ldx) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  if (n < 1 || nrhs < 0 || lda < n || ldx < n) return fail(h, MIQR_EINVAL, "bad sizes");
  if (bad_ptr(VR) || bad_ptr(X)) return fail(h, MIQR_EINVAL, "null pointer");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  find_zero_diagonal(s, n, VR, lda, h->dflag);
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, h->dflag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(h, e, "qr_solve_r");
  if (flag) return fail(h, MIQR_ESINGULAR, "R(" + std::to_string(flag - 1) + ") == 0");
  if (nrhs == 0) return MIQR_OK;
  const int64_t scratch_n = int64_t(4) << 20;
  miqr_status st = ensure_ws(h, (size_t)(scratch_n + 64) * sizeof(double));
  if (st != MIQR_OK) return st;
  e = solve_upper(s, n, nrhs, VR, lda, X, ldx, (double*)h->ws, scratch_n);
  if (e != hipSuccess) return hip_fail(h, e, "qr_solve_r");
  return MIQR_OK;
}

miqr_status qr_backward_error(miqr_handle h, void* stream, int64_t m, int64_t n, int64_t nrhs,
                              const double* A, int64_t lda, const double* B, int64_t ldb,
                              const double* X, int64_t ldx, double* beta) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (n < 1 || m < n || nrhs < 1) return fail(h, MIQR_EINVAL, "need m >= n >= 1, nrhs >= 1");
  if (lda < m || ldb < m || ldx < n) return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(A) || bad_ptr(B) || bad_ptr(X) || bad_ptr(beta))
    return fail(h, MIQR_EINVAL, "null pointer");
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  const int64_t scn = int64_t(4) << 20;
  double *Rr = nullptr, *U = nullptr, *nrm = nullptr, *sc = nullptr;
  auto carve = [&](Arena& ar) {
    Rr = ar.take(m * nrhs);
    U = ar.take(n * nrhs);
    nrm = ar.take(3 * nrhs + n + 8);
    sc = ar.take(scn);
  };
  Arena dry{nullptr};
  carve(dry);
  miqr_status st = ensure_ws(h, (size_t)dry.off * sizeof(double));
  if (st != MIQR_OK) return st;
  Arena ar{(double*)h->ws};
  carve(ar);
  hipError_t e = hipSuccess;
  backward_error_dev((hipStream_t)stream, m, n, nrhs, A, lda, B, ldb, X, ldx, Rr, U, nrm, sc, scn,
                     &e, beta);
  if (e != hipSuccess) return hip_fail(h, e, "qr_backward_error");
  return MIQR_OK;
}

miqr_status qr_lstsq(miqr_handle h, void* stream, int64_t m, int64_t n, int64_t nrhs, double* A,
                     int64_t lda, double* B, int64_t ldb, const qr_opts* o, qr_info* info) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (n < 1 || m < n || nrhs < 1) return fail(h, MIQR_EINVAL, "need m >= n >= 1, nrhs >= 1");
  if (lda < m || ldb < m) return fail(h, MIQR_EINVAL, "leading dimension too small");
  if (bad_ptr(A) || bad_ptr(B)) return fail(h, MIQR_EINVAL, "null pointer");
  const int prec = o ? o->precision : MIQR_FP64;
  if (prec != MIQR_FP64 && prec != MIQR_MIXED_FP32 && prec != MIQR_MIXED_BF16)
    return fail(h, MIQR_EINVAL, "bad precision");
  if (o && (o->normalize || o->Q)) return fail(h, MIQR_ENOTSUP, "lstsq takes no Q/normalize");
  miqr_status cst = check_opts(h, m, o);
  if (cst != MIQR_OK) return cst;
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  if (info) std::memset(info, 0, sizeof(*info));
  if (prec != MIQR_FP64) {
    const int comp = prec == MIQR_MIXED_FP32 ? COMPUTE_F32 : COMPUTE_BF16;
    return lstsq_mixed(h, s, m, n, nrhs, A, lda, B, ldb, o, comp, info);
  }

  // Layout: the factorisation's regions first, then T, W1, W2, and (for
  // info) the originals and the residual.
  const Tuning tune = tuning_for(h, m, n, o, true);
  const FactorLayout L = factor_layout(m, n, tune);
  const int64_t tr = t_rows(tune, n);
  FactorWs f;
  double *T = nullptr, *W1 = nullptr, *W2 = nullptr;
  double *A0 = nullptr, *B0 = nullptr, *Rr = nullptr, *nrm = nullptr;
  auto carve = [&](double* base) {
    f = carve_factor(base, L);
    Arena ar{base};
    ar.off = f.doubles;
    T = ar.take(tr * n);
    W1 = ar.take(n * nrhs);
    W2 = ar.take(n * nrhs);
    if (info) {
      A0 = ar.take(m * n);
      B0 = ar.take(m * nrhs);
      Rr = ar.take(m * nrhs);
      nrm = ar.take(3 * nrhs + n + 8);
    }
    return ar.off;
  };
  const int64_t need = carve(nullptr);
  miqr_status st = ensure_ws(h, (size_t)need * sizeof(double));
  if (st != MIQR_OK) return st;
  carve((double*)h->ws);
  if (info) {
    copy_matrix(s, m, n, A, lda, A0, m);
    copy_matrix(s, m, nrhs, B, ldb, B0, m);
  }
  st = lstsq_core(h, s, tune, f, m, n, nrhs, A, lda, B, ldb, T, W1, W2, info);
  if (st != MIQR_OK) return st;
  if (info) {
    hipError_t e = hipSuccess;
    info->backward_error = backward_error_dev(s, m, n, nrhs, A0, m, B0, m, B, ldb, Rr, W1, nrm,
                                              f.scratch, f.scratch_n, &e);
    if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq info");
  }
  return MIQR_OK;
}

miqr_status qr_lstsq_batched_ex(miqr_handle h, void* stream, int64_t count,
                                const qr_batch_item* items, const qr_opts* o, int32_t* status,
                                int32_t* iters) {
  if (!h) return MIQR_EINVAL;
  ProfScope prof_scope(h);
  h->err.clear();
  if (count < 0 || count > (int64_t)1 << 30 || (count > 0 && !items))
    return fail(h, MIQR_EINVAL, "bad count or items");
  const int precision = o ? o->precision : MIQR_FP64;
  if (precision != MIQR_FP64 && precision != MIQR_MIXED_FP32 && precision != MIQR_MIXED_BF16)
    return fail(h, MIQR_EINVAL, "unknown precision");
  const int prec = precision == MIQR_MIXED_FP32   ? kBlkF32
                   : precision == MIQR_MIXED_BF16 ? kBlkBF16
                                                  : kBlkF64;
  if (o && (o->normalize || o->Q)) return fail(h, MIQR_ENOTSUP, "batched lstsq takes no Q/normalize");
  int64_t rtot = 0;  // R (n x n) and C (n x nrhs) per problem, each 32-double aligned
  double bytes = 0.0, flops = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    const qr_batch_item& it = items[i];
    const std::string at = " (item " + std::to_string(i) + ")";
    if (it.n < 1 || it.m < it.n || it.m > INT32_MAX)
      return fail(h, MIQR_EINVAL, "need 2^31 > m >= n >= 1" + at);
    if (it.nrhs < 1 || it.nrhs > kBatchMaxRhs)
      return fail(h, MIQR_EINVAL, "need 1 <= nrhs <= " + std::to_string(kBatchMaxRhs) + at);
    if (it.n + it.nrhs > kBatchMaxCols)
      return fail(h, MIQR_EINVAL, "need n + nrhs <= " + std::to_string(kBatchMaxCols) + at);
    if (it.lda < it.m || it.ldb < it.m) return fail(h, MIQR_EINVAL, "leading dimension too small" + at);
    if (bad_ptr(it.A) || bad_ptr(it.B)) return fail(h, MIQR_EINVAL, "null pointer" + at);
    rtot += ((it.n * it.n + 31) & ~int64_t(31)) + ((it.n * it.nrhs + 31) & ~int64_t(31));
    batch_item_cost(it, &bytes, &flops);
  }
  if (count == 0) return MIQR_OK;
  if (hipSetDevice(h->device) != hipSuccess) return fail(h, MIQR_EHIP, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int64_t task_d = ((int64_t)batch_table_bytes(count) + 255) / 256 * 32;
  const int64_t stat_d = (2 * count * 4 + 255) / 256 * 32;
  miqr_status st = ensure_ws(h, (size_t)(task_d + stat_d + 32 + rtot) * sizeof(double));
  if (st != MIQR_OK) return st;
  st = ensure_pinned(h, count);
  if (st != MIQR_OK) return st;
  Arena ar{(double*)h->ws};
  BatchHeader* dtable = (BatchHeader*)ar.take(task_d);
  int* dstatus = (int*)ar.take(stat_d);
  int* diters = dstatus + count;
  int* counter = (int*)ar.take(32);
  double* rbase = ar.take(rtot);
  std::vector<int64_t> roff((size_t)count);
  for (int64_t i = 0, off = 0; i < count; ++i) {
    roff[(size_t)i] = off;
    off += ((items[i].n * items[i].n + 31) & ~int64_t(31)) +
           ((items[i].n * items[i].nrhs + 31) & ~int64_t(31));
  }
  // Enqueue the items of `sel` in precision p: tasks grouped by queue (the
  // refinement kernel takes queues 1..3 as one contiguous range), largest
  // problems first within each queue (their cost is about blocks x columns^2
  // steps), so that every persistent grid ends with small problems.
  auto launch = [&](const std::vector<int64_t>& sel, int p) -> miqr_status {
    st = ensure_pinned(h, (int64_t)sel.size());
    if (st != MIQR_OK) return st;
    std::vector<BatchTask> tk(sel.size());
    std::vector<int> q(sel.size());
    for (size_t k = 0; k < sel.size(); ++k) {
      const int64_t i = sel[k];
      const qr_batch_item& it = items[i];
      BatchTask& t = tk[k];
      t = BatchTask{};
      t.A = it.A;
      t.B = it.B;
      t.R = rbase + roff[(size_t)i];
      t.C = t.R + ((it.n * it.n + 31) & ~int64_t(31));
      t.lda = it.lda;
      t.ldb = it.ldb;
      t.m = (int)it.m;
      t.n = (int)it.n;
      t.nrhs = (int)it.nrhs;
      t.flags = kTaskWriteR;
      t.slot = (int)i;
      q[k] = batch_queue(t);
    }
    std::vector<size_t> order(sel.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = k;
    auto cost = [&](size_t k) {
      const double N = (double)tk[k].n + tk[k].nrhs;
      return ((tk[k].m + kBatchRows - 1) / kBatchRows + 1) * N * N;
    };
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
      return q[a] != q[b] ? q[a] < q[b] : cost(a) > cost(b);
    });
    BatchHeader* hd = h->pin_tasks;
    *hd = BatchHeader{};
    BatchTask* pt = batch_tasks(hd);
    hd->total = (int)sel.size();
    for (size_t k = 0; k < order.size(); ++k) {
      pt[k] = tk[order[k]];
      hd->count[q[order[k]]]++;
    }
    for (int k = 1; k < kBatchQueues; ++k) hd->begin[k] = hd->begin[k - 1] + hd->count[k - 1];
    hipError_t e = hipMemcpyAsync(dtable, hd, batch_table_bytes((int64_t)sel.size()),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(h->table_ev, s);
    if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq_batched upload");
    BatchGrids g = batched_grids(h->device, p);
    for (int k = 0; k < kBatchQueues; ++k) g.g[k] = std::min(g.g[k], hd->count[k]);
    g.g[kBatchQueues] = std::min<int64_t>(g.g[kBatchQueues], (int64_t)sel.size());
    batched_ls(s, dtable, counter, dstatus, diters, g, p, bytes, flops);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq_batched launch");
    return MIQR_OK;
  };
  auto fetch = [&]() -> miqr_status {
    hipError_t e = hipMemcpyAsync(h->pin_status, dstatus, 2 * count * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "qr_lstsq_batched status");
    return MIQR_OK;
  };
  std::vector<int64_t> all((size_t)count);
  for (int64_t i = 0; i < count; ++i) all[(size_t)i] = i;
  st = launch(all, prec);
  if (st != MIQR_OK) return st;
  if (!status && !iters && prec == kBlkF64) return MIQR_OK;
  st = fetch();
  if (st != MIQR_OK) return st;
  std::vector<int32_t> stv(h->pin_status, h->pin_status + count);
  std::vector<int32_t> itv((size_t)count, 0);
  if (prec != kBlkF64) {
    // Problems whose refinement missed the target are solved again in FP64
    // (their A and B were left as they were).
    std::vector<int64_t> redo;
    for (int64_t i = 0; i < count; ++i) {
      itv[(size_t)i] = h->pin_status[count + i];
      if (stv[(size_t)i] == kStatusNoConv) redo.push_back(i);
    }
    if (!redo.empty()) {
      st = launch(redo, kBlkF64);
      if (st != MIQR_OK) return st;
      st = fetch();
      if (st != MIQR_OK) return st;
      for (int64_t i : redo) {
        stv[(size_t)i] = h->pin_status[i];
        itv[(size_t)i] = -1;
      }
    }
  }
  int64_t bad = -1;
  for (int64_t i = 0; i < count; ++i) {
    if (status) status[i] = stv[(size_t)i];
    if (iters) iters[i] = itv[(size_t)i];
    if (stv[(size_t)i] != 0 && bad < 0) bad = i;
  }
  for (int64_t i = 0; i < count; ++i)
    if (stv[(size_t)i] == kStatusFault)
      return fail(h, MIQR_EHIP, "item " + std::to_string(i) + ": batched kernel wait bound reached");
  if (bad >= 0)
    return fail(h, MIQR_ESINGULAR, "item " + std::to_string(bad) + ": R(" +
                                       std::to_string(stv[(size_t)bad] - 1) + ") == 0");
  return MIQR_OK;
}

miqr_status qr_lstsq_batched(miqr_handle h, void* stream, int64_t count,
                             const qr_batch_item* items, const qr_opts* o, int32_t* status) {
  return qr_lstsq_batched_ex(h, stream, count, items, o, status, nullptr);
}

}  // extern "C"

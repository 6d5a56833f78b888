// Host-side planning: tuning, split rule, workspace layout and the cost
// model that chooses the tuning.  Pure host code; nothing here touches a
// device.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "common.h"
#include "tsqr.h"

namespace miqr {

TsqrGeom tsqr_geometry(int64_t rows, int w, int leaf_rows, int chain, int arity) {
  TsqrGeom g;
  if (leaf_rows != 128 && leaf_rows != 256) leaf_rows = (rows >= 256 * 64) ? 256 : 128;
  g.leaf_rows = leaf_rows;
  g.blocks = std::max<int64_t>(1, (rows + leaf_rows - 1) / leaf_rows);
  // Default chains leave about 512 of them (two workgroups per CU for the
  // stacked-block launch), at most eight blocks each.
  if (chain <= 0) chain = (int)std::max<int64_t>(1, std::min<int64_t>(8, g.blocks / 512));
  g.chain = chain;
  // A tree node stacks arity - 1 child R factors (w rows each) in kYL rows.
  const int max_arity = 1 + kYL / std::max(w, 1);
  if (arity < 2) arity = std::min(max_arity, 5);
  g.arity = std::min(arity, max_arity);
  g.chains = (g.blocks + chain - 1) / chain;
  int64_t nodes = g.chains;
  while (nodes > 1 && g.levels < kMaxLevels - 1) {
    nodes = (nodes + g.arity - 1) / g.arity;
    g.tree_nodes += nodes;
    ++g.levels;
  }
  return g;
}

int64_t eg_split(int64_t nk, const Tuning& t) {
  if (nk <= t.bstar) return 0;
  // Alg. 2 splits at floor(n/2); any split gives the same factors in exact
  // arithmetic.  Rounding the left width up to a multiple of the threshold
  // keeps panels full width and GEMM operands aligned.
  const int64_t unit = nk > t.b ? t.b : t.bstar;
  int64_t n1 = ((nk / 2 + unit - 1) / unit) * unit;
  if (n1 >= nk) n1 = nk / 2;
  return std::max<int64_t>(n1, 1);
}

namespace {

// Largest n1 x n2 product (M1 .. M4 of Alg. 2) over every node of the
// recursion of a width-nk problem.  The root's is not always the largest: for
// nk in [2b + 2, 2.5b) the left child is 2b wide and splits into b x b, more
// than the root's n1 x n2.
int64_t max_node_product(int64_t nk, const Tuning& t) {
  const int64_t n1 = eg_split(nk, t);
  if (n1 == 0) return 0;
  return std::max(n1 * (nk - n1),
                  std::max(max_node_product(n1, t), max_node_product(nk - n1, t)));
}

// TSQR workspace of one panel, in doubles (tsqr_plan's own slot layout).
int64_t tsqr_ws(int64_t rows, int w, const Tuning& t) {
  int lr = t.leaf_rows, ch = t.chain, ar = t.arity;
  if (lr == 0 || ch == 0 || ar == 0) {
    int a = 0, b = 0, c = 0;
    tsqr_auto(rows, w, &a, &b, &c);
    if (lr == 0) lr = a;
    if (ch == 0) ch = b;
    if (ar == 0) ar = c;
  }
  return tsqr_plan(rows, w, lr, ch, ar, nullptr).workspace_doubles;
}

// Largest TSQR workspace over the panels of a width-nk problem starting at
// mk rows.
void max_panel_ws(int64_t mk, int64_t nk, const Tuning& t, int64_t* best) {
  const int64_t n1 = eg_split(nk, t);
  if (n1 == 0) {
    *best = std::max(*best, tsqr_ws(mk, (int)nk, t));
    return;
  }
  max_panel_ws(mk, n1, t, best);
  max_panel_ws(mk - n1, nk - n1, t, best);
}

int64_t top_panel(const Tuning& t, int64_t n) {
  return t.t_layout == T_BLOCKED ? std::min<int64_t>(std::max<int64_t>(t.nb, 1), n) : n;
}

}  // namespace

FactorLayout factor_layout(int64_t m, int64_t n, const Tuning& t, bool with_q) {
  FactorLayout L;
  const int64_t nb = top_panel(t, n);
  // Every top-level panel is a width-nb problem (the last may be narrower).
  for (int64_t j = 0; j < n; j += nb) {
    const int64_t w = std::min(nb, n - j);
    max_panel_ws(m - j, w, t, &L.tsqr);
    L.wa = std::max(L.wa, max_node_product(w, t));
  }
  L.wa = std::max<int64_t>(L.wa, 1);
  L.wb = L.wa;
  // Split-K partials: room for 512 splits of a 128 x 128 product.
  L.scratch = std::max<int64_t>(int64_t(8) << 20, 4 * L.wa);
  if (t.t_layout == T_BLOCKED && nb < n) {
    L.u1 = nb * nb;
    L.u2 = nb * nb;
    L.scratch = std::max<int64_t>(L.scratch, 4 * nb * nb);
    const int64_t rest = nb * std::max<int64_t>(n - nb, 1);
    L.ua1 = rest;
    L.ua2 = rest;
    L.scratch_aux = std::max<int64_t>(int64_t(8) << 20, 2 * rest);
  }
  if (with_q && n > t.bstar) {
    // FULL: W = T V_top^T (n x n); BLOCKED: one panel's V^T Q (nb x n).
    const int64_t q = (t.t_layout == T_BLOCKED ? nb : n) * n;
    L.ua1 = std::max(L.ua1, q);
    L.ua2 = std::max(L.ua2, q);
    L.scratch_aux = std::max<int64_t>(L.scratch_aux, int64_t(8) << 20);
  }
  auto al = [](int64_t v) { return (v + 31) & ~int64_t(31); };
  L.total = al(L.tsqr) + al(L.wa) + al(L.wb) + al(L.scratch) + al(L.u1) + al(L.u2) + al(L.ua1) +
            al(L.ua2) + al(L.scratch_aux) + 128;
  return L;
}

// ------------------------------------------------------------ cost model

const char* cost_feature_name(int f) {
  static const char* names[F_COUNT] = {"leaf256_steps", "leaf128_steps", "tree_levels",
                                       "tree_levels_small", "hr", "down_levels",
                                       "gemm_launches", "gemm_flops", "gemm_flops_per_depth",
                                       "gemm_idle_flops", "panel_bytes"};
  return (f >= 0 && f < F_COUNT) ? names[f] : "";
}

const CostCoeffs& cost_coeffs() {
  // Fitted by least squares to factorisations timed on MI355X over a sweep of
  // shapes and tunings, one stream, no look-ahead (the fit and its residuals
  // are kept with the measured profiles); d0 from the GEMM depth scan.
  static const CostCoeffs c{
      {
          /*leaf256_steps=*/0.0001165,
          /*leaf128_steps=*/0.0001088,
          /*tree_levels=*/0.0001303,
          /*tree_levels_small=*/8.415e-05,
          /*hr=*/3.599e-05,
          /*down_levels=*/0,
          /*gemm_launches=*/2.788e-06,
          /*gemm_flops=*/1.754e-14,
          /*gemm_flops_per_depth=*/3.549e-13,
          /*gemm_idle_flops=*/4.973e-14,
          /*panel_bytes=*/2.579e-13,
      },
      /*overlap=*/0.99,
  };
  return c;
}

namespace {

struct Feat {
  double f[F_COUNT] = {};
  double seconds() const {
    const CostCoeffs& c = cost_coeffs();
    double s = 0.0;
    for (int i = 0; i < F_COUNT; ++i) s += c.c[i] * f[i];
    return s;
  }
  void add(const Feat& o) {
    for (int i = 0; i < F_COUNT; ++i) f[i] += o.f[i];
  }
};

struct Acc {
  CostEstimate e;
};

Feat tsqr_feat(int64_t rows, int w, int lr, int ch, int ar, bool with_q) {
  Feat r;
  const TsqrGeom g = tsqr_geometry(rows, w, lr, ch, ar);
  // Leaf: the first block of every chain in one launch (one workgroup per
  // CU at 256-row blocks, two at 128), then the stacked blocks (two per CU).
  const double slots1 = g.leaf_rows == 256 ? 256.0 : 512.0;
  const double waves1 = std::ceil((double)g.chains / slots1);
  const double waves2 = std::ceil((double)g.chains / 512.0);
  r.f[g.leaf_rows == 256 ? F_LEAF256 : F_LEAF128] = waves1 + (g.chain - 1) * waves2;
  // Tree nodes stack (arity - 1) R factors: above 128 rows they run on the
  // blocked MFMA node kernel, up to 128 on the column-by-column one.
  r.f[(g.arity - 1) * w > 128 ? F_TREE : F_TREE_SMALL] = g.levels;
  r.f[F_HR] = 1.0;
  r.f[F_DOWN] = g.levels + 1;
  r.f[F_BYTES] = 8.0 * (double)rows * w * (with_q ? 5.0 : 4.0);
  return r;
}

// The workgroups the GEMM dispatch launches for an M x N x K product (its
// tile and split-K rule): a product with fewer than one per CU runs at that
// share of the chip.
double gemm_units(double M, double N, double K, bool* split) {
  const double t128 = std::ceil(M / 128.0) * std::ceil(N / 128.0);
  const bool big = M >= 128 && N >= 128 && (t128 >= 128 || K >= 4096);
  const double bm = big ? 128.0 : 64.0;
  const double tiles = std::ceil(M / bm) * std::ceil(N / bm);
  double nsplit = 1.0;
  const double min_chunk = K >= 1024 ? 512.0 : 32.0;
  if (tiles < 512 && K >= 2 * min_chunk)
    nsplit = std::max(1.0, std::min(std::floor((1024 + tiles - 1) / tiles), std::floor(K / min_chunk)));
  *split = nsplit > 1.0;
  return tiles * nsplit;
}

Feat gemm_feat(double M, double N, double K, Acc* acc) {
  Feat r;
  const double fl = 2.0 * M * N * K;
  bool split = false;
  const double units = gemm_units(M, N, K, &split);
  const double d = std::max(1.0, std::min({M, N, K}));
  r.f[F_GEMM_LAUNCH] = split ? 2.0 : 1.0;  // with the split-K reduce
  r.f[F_GEMM_FLOP] = fl;
  r.f[F_GEMM_DEPTH] = fl / d;
  r.f[F_GEMM_IDLE] = fl * std::max(0.0, 256.0 / std::max(units, 1.0) - 1.0);
  if (acc) acc->e.gemm_flops += fl;
  return r;
}

// Alg. 2 on a width-nk problem of mk rows, all on one stream.
Feat eg_feat(int64_t mk, int64_t nk, const Tuning& t, bool with_q, bool spine_t, bool spine,
             Acc* acc) {
  const int64_t n1 = eg_split(nk, t);
  if (n1 == 0) {
    int lr = t.leaf_rows, ch = t.chain, ar = t.arity;
    int a = 0, b = 0, c = 0;
    tsqr_auto(mk, (int)nk, &a, &b, &c);
    if (acc) acc->e.panels += 1;
    return tsqr_feat(mk, (int)nk, lr ? lr : a, ch ? ch : b, ar ? ar : c, with_q);
  }
  const int64_t n2 = nk - n1;
  Feat s = eg_feat(mk, n1, t, false, true, false, acc);
  s.add(gemm_feat(n1, n2, mk, acc));
  s.add(gemm_feat(n1, n2, n1, acc));
  s.add(gemm_feat(mk, n2, n1, acc));
  s.add(eg_feat(mk - n1, n2, t, false, spine_t, spine, acc));
  if (!spine || spine_t) {
    s.add(gemm_feat(n1, n2, mk - n1, acc));
    s.add(gemm_feat(n1, n2, n2, acc));
    s.add(gemm_feat(n1, n2, n1, acc));
  }
  return s;
}

// Top-level update of panel (rows mk, width w) on ncols columns.
Feat update_feat(int64_t mk, int64_t w, int64_t ncols, Acc* acc) {
  Feat s;
  if (ncols <= 0) return s;
  s.add(gemm_feat(w, ncols, mk, acc));
  s.add(gemm_feat(w, ncols, w, acc));
  s.add(gemm_feat(mk, ncols, w, acc));
  return s;
}

}  // namespace

static CostEstimate predict_impl(int64_t m, int64_t n, const Tuning& t, bool lstsq) {
  Acc acc;
  Feat tot;
  double s = 0.0;
  if (t.t_layout != T_BLOCKED) {
    tot = eg_feat(m, n, t, false, !lstsq, true, &acc);
    s = tot.seconds();
    acc.e.critical_s = s;
  } else {
    const int64_t nb = top_panel(t, n);
    std::vector<double> F, Un, Ur;
    for (int64_t j = 0; j < n; j += nb) {
      const int64_t w = std::min(nb, n - j);
      const Feat fp = eg_feat(m - j, w, t, false, true, false, &acc);
      const int64_t nxt = std::min(nb, std::max<int64_t>(n - j - w, 0));
      const Feat un = update_feat(m - j, w, nxt, &acc);
      const Feat ur = update_feat(m - j, w, n - j - w - nxt, &acc);
      F.push_back(fp.seconds());
      Un.push_back(un.seconds());
      Ur.push_back(ur.seconds());
      acc.e.schedule.push_back({fp.f, un.f, ur.f});
      tot.add(fp);
      tot.add(un);
      tot.add(ur);
    }
    double crit = 0.0, upd = 0.0;
    for (double f : F) crit += f;
    for (size_t k = 0; k < F.size(); ++k) upd += Un[k] + Ur[k];
    acc.e.critical_s = crit;
    acc.e.update_s = upd;
    if (t.lookahead) {
      const double ov = cost_coeffs().overlap;
      s = F[0];
      for (size_t k = 0; k + 1 < F.size(); ++k) {
        const double a = Un[k] + F[k + 1], b = Ur[k];
        s += std::max(a, b) + ov * std::min(a, b);
      }
    } else {
      s = tot.seconds();
    }
  }
  for (int i = 0; i < F_COUNT; ++i) acc.e.f[i] = tot.f[i];
  acc.e.seconds = s;
  return acc.e;
}

CostEstimate predict(int64_t m, int64_t n, const Tuning& t) { return predict_impl(m, n, t, false); }

void tsqr_auto(int64_t rows, int w, int* leaf_rows, int* chain, int* arity) {
  // Memoised argmin of the panel cost over the block height, chain length and
  // tree arity, per (rows, width).
  static std::mutex mu;
  static std::map<std::pair<int64_t, int>, std::tuple<int, int, int>> memo;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find({rows, w});
    if (it != memo.end()) {
      std::tie(*leaf_rows, *chain, *arity) = it->second;
      return;
    }
  }
  double best = 1e300;
  int bl = 0, bc = 0, ba = 0;
  const int max_arity = 1 + kYL / std::max(w, 1);
  for (int lr : {128, 256}) {
    // 256-row blocks only where there are at least two full ones.
    if (lr == 256 && rows < 512) continue;
    const int64_t P0 = std::max<int64_t>(1, (rows + lr - 1) / lr);
    for (int ch : {1, 2, 4, 8}) {
      if (ch > 1 && ch > P0) continue;
      // The tree arity stays at five stacked children (or what the stacked-R
      // buffer holds for narrower panels): in the sweep, narrower trees lost
      // wherever they were measured against it, and the per-level costs of
      // the two node kernels are not separable from the other per-panel
      // terms in the fit.
      for (int ar : {std::min(5, max_arity)}) {
        const double s = tsqr_feat(rows, w, lr, ch, ar, false).seconds();
        if (s < best * (1.0 - 1e-9)) {
          best = s;
          bl = lr;
          bc = ch;
          ba = ar;
        }
      }
    }
  }
  *leaf_rows = bl;
  *chain = bc;
  *arity = ba;
  std::lock_guard<std::mutex> g(mu);
  if (memo.size() > 65536) memo.clear();
  memo[{rows, w}] = std::make_tuple(bl, bc, ba);
}

Tuning choose_tuning(int64_t m, int64_t n, const qr_opts* o, bool lstsq) {
  Tuning t;
  int64_t b = 0, bstar = 0, nb = 0;
  int layout = lstsq ? -1 : T_FULL;  // -1: least squares picks the layout
  if (o) {
    b = o->b;
    bstar = o->bstar;
    nb = o->nb;
    t.leaf_rows = (int)o->leaf_rows;
    t.chain = (int)o->chain;
    t.arity = o->arity >= 2 ? (int)o->arity : 0;
    if (!lstsq) layout = o->t_layout;
    else if (o->t_layout == T_BLOCKED) layout = T_BLOCKED;
    t.lookahead = o->no_lookahead ? 0 : 1;
  }
  // Candidates for what the caller left open.
  std::vector<int64_t> bs = b > 0 ? std::vector<int64_t>{b} : std::vector<int64_t>{32, 64, 128};
  std::vector<int64_t> bss;
  if (bstar > 0) bss = {bstar};
  else if (b > 0) bss = {std::min<int64_t>(b, kNB)};
  else bss = {32, 64};
  std::vector<int64_t> nbs = nb > 0 ? std::vector<int64_t>{nb}
                                    : std::vector<int64_t>{128, 256, 512, 1024};
  std::vector<int> layouts = layout >= 0 ? std::vector<int>{layout}
                                         : std::vector<int>{T_FULL, T_BLOCKED};
  double best = 1e300;
  Tuning pick = t;
  for (int lay : layouts)
    for (int64_t bb : bs)
      for (int64_t bsv : bss) {
        if (bsv > bb || bsv > kNB) continue;
        for (int64_t nbv : (lay == T_BLOCKED ? nbs : std::vector<int64_t>{0})) {
          Tuning c = t;
          c.t_layout = lay;
          c.b = std::min<int64_t>(bb, std::max<int64_t>(n, 1));
          c.bstar = (int)std::min<int64_t>(bsv, std::max<int64_t>(n, 1));
          if (c.b < c.bstar) c.b = c.bstar;
          c.nb = lay == T_BLOCKED ? std::min<int64_t>(nbv, n) : 0;
          if (lay == T_BLOCKED && c.nb < c.bstar) continue;
          const double s = predict_impl(m, n, c, lstsq).seconds;
          if (s < best * (1.0 - 1e-9)) {
            best = s;
            pick = c;
          }
        }
      }
  if (best == 1e300) {
    // Only reachable with caller values the entry points reject first.
    pick.b = std::max<int64_t>(1, std::min<int64_t>(b > 0 ? b : 64, n));
    pick.bstar = (int)std::min<int64_t>(pick.b, kNB);
    pick.t_layout = layout >= 0 ? layout : T_FULL;
    pick.nb = pick.t_layout == T_BLOCKED ? std::min<int64_t>(nb > 0 ? nb : 512, n) : 0;
  }
  return pick;
}

namespace {
void list_nodes(int64_t c0, int64_t mk, int64_t nk, const Tuning& t, std::string* out,
                bool* first) {
  const int64_t n1 = eg_split(nk, t);
  char buf[96];
  std::snprintf(buf, sizeof buf, "%s[%lld,%lld,%lld,%lld]", *first ? "" : ",", (long long)c0,
                (long long)mk, (long long)nk, (long long)n1);
  *first = false;
  *out += buf;
  if (n1 == 0) return;
  list_nodes(c0, mk, n1, t, out, first);
  list_nodes(c0 + n1, mk - n1, nk - n1, t, out, first);
}
}  // namespace

std::string describe_plan(int64_t m, int64_t n, const Tuning& t) {
  const FactorLayout L = factor_layout(m, n, t);
  const CostEstimate e = predict(m, n, t);
  std::string s;
  char buf[1024];
  std::snprintf(buf, sizeof buf,
                "{\"m\":%lld,\"n\":%lld,\"tuning\":{\"b\":%lld,\"bstar\":%d,\"nb\":%lld,"
                "\"leaf_rows\":%d,\"chain\":%d,\"arity\":%d,\"t_layout\":%d,\"lookahead\":%d},"
                "\"cost\":{\"seconds\":%.9g,\"panels\":%lld,\"gemm_flops\":%.9g,"
                "\"critical_s\":%.9g,\"update_s\":%.9g},"
                "\"layout\":{\"tsqr\":%lld,\"wa\":%lld,\"wb\":%lld,\"scratch\":%lld,\"u1\":%lld,"
                "\"u2\":%lld,\"ua1\":%lld,\"ua2\":%lld,\"scratch_aux\":%lld,\"total\":%lld},",
                (long long)m, (long long)n, (long long)t.b, t.bstar, (long long)t.nb, t.leaf_rows,
                t.chain, t.arity, t.t_layout, t.lookahead, e.seconds, (long long)e.panels,
                e.gemm_flops, e.critical_s, e.update_s, (long long)L.tsqr,
                (long long)L.wa, (long long)L.wb, (long long)L.scratch, (long long)L.u1,
                (long long)L.u2, (long long)L.ua1, (long long)L.ua2, (long long)L.scratch_aux,
                (long long)L.total);
  s += buf;
  // The cost model's features (one-stream counts) and coefficients.
  s += "\"features\":{";
  for (int i = 0; i < F_COUNT; ++i) {
    std::snprintf(buf, sizeof buf, "%s\"%s\":%.9g", i ? "," : "", cost_feature_name(i), e.f[i]);
    s += buf;
  }
  s += "},\"schedule\":[";
  // BLOCKED: per top-level panel, the features of its factorisation, of the
  // update of the next panel's columns and of the rest of the update.
  for (size_t k = 0; k < e.schedule.size(); ++k) {
    s += k ? ",[" : "[";
    for (int part = 0; part < 3; ++part) {
      s += part ? ",[" : "[";
      for (int i = 0; i < F_COUNT; ++i) {
        std::snprintf(buf, sizeof buf, "%s%.9g", i ? "," : "", e.schedule[k].part[part][i]);
        s += buf;
      }
      s += "]";
    }
    s += "]";
  }
  s += "],\"coefficients\":{";
  for (int i = 0; i < F_COUNT; ++i) {
    std::snprintf(buf, sizeof buf, "%s\"%s\":%.9g", i ? "," : "", cost_feature_name(i),
                  cost_coeffs().c[i]);
    s += buf;
  }
  std::snprintf(buf, sizeof buf, ",\"overlap\":%.9g},", cost_coeffs().overlap);
  s += buf;
  // Recursion nodes [c0, rows, width, n1] (n1 = 0: base-case TSQR panel) of
  // every top-level panel.
  s += "\"nodes\":[";
  bool first = true;
  const int64_t nb = top_panel(t, n);
  for (int64_t j = 0; j < n; j += nb) list_nodes(j, m - j, std::min(nb, n - j), t, &s, &first);
  s += "],\"panels\":[";
  first = true;
  // TSQR geometry of each base-case panel.
  std::vector<std::tuple<int64_t, int64_t, int64_t>> leaves;
  struct W {
    static void walk(int64_t c0, int64_t mk, int64_t nk, const Tuning& t,
                     std::vector<std::tuple<int64_t, int64_t, int64_t>>* v) {
      const int64_t n1 = eg_split(nk, t);
      if (n1 == 0) {
        v->emplace_back(c0, mk, nk);
        return;
      }
      walk(c0, mk, n1, t, v);
      walk(c0 + n1, mk - n1, nk - n1, t, v);
    }
  };
  for (int64_t j = 0; j < n; j += nb) W::walk(j, m - j, std::min(nb, n - j), t, &leaves);
  for (auto& lf : leaves) {
    int64_t c0, mk, nk;
    std::tie(c0, mk, nk) = lf;
    int a = 0, b = 0, c = 0;
    tsqr_auto(mk, (int)nk, &a, &b, &c);
    const TsqrGeom g = tsqr_geometry(mk, (int)nk, t.leaf_rows ? t.leaf_rows : a,
                                     t.chain ? t.chain : b, t.arity ? t.arity : c);
    std::snprintf(buf, sizeof buf, "%s[%lld,%lld,%lld,%d,%d,%d,%d]", first ? "" : ",",
                  (long long)c0, (long long)mk, (long long)nk, g.leaf_rows, g.chain, g.arity,
                  g.levels);
    first = false;
    s += buf;
  }
  s += "]}";
  return s;
}

}  // namespace miqr

// stats.cpp -- the PP-STAT statistics as fixed sequences of CKKS operations.
//
// Paper references: Mean(x,B) and Variance(x,B) with pre-normalisation
// scaling (Sec. 5.1, Eq. 2); CryptoInvSqrt = Chebyshev initial value
// (Alg. 3, Eq. 3) + Newton iterations (Alg. 2); ZNorm (Alg. 4); kurtosis
// (Alg. 5) and skewness (its mirror, Sec. 5); CV (Alg. 6); PCC (Sec. 5.5).
//
// Conventions that make the sequence reproducible bit for bit:
//   * a binary operation on operands at different levels first brings the
//     higher one down to the lower level (level_align);
//   * sums over lists fold left to right;
//   * FP64 constants are formed exactly as written below;
//   * Newton (n = 2) runs in the balanced order y2 = y*y, p1 = w2*y,
//     p2 = p1*y2, y = 1.5 y - p2 with w2 = (B'/2) v, two levels per step;
//   * sqrt(v; B') = 2 * w2 * InvSqrt(v; B') (Alg. 6 reads CryptoSqrt(var, B);
//     with Variance(x,B) = Var/B^2 the factor has to be B^2);
//   * PCC = Cov * InvSqrt(Var x; Bx^2) * InvSqrt(Var y; By^2);
//   * slots past the row count are zero; centred moments use a 1/n row mask,
//     a constant when a ciphertext is full and a plaintext vector otherwise.
#include "stats.h"

#include "boot.h"

#include <future>
#include <map>
#include <tuple>

#include <map>
#include <tuple>
#include <cmath>

namespace ppst {

namespace {

struct Circ {
  Context& cx;
  const EvalKeys& evk;
  // embedding of a ragged column's row mask, computed on a host thread while
  // the device runs the circuit up to mask_mean (see prefetch_mask)
  size_t mask_rows = 0, mask_n = 0;
  std::shared_future<std::vector<long double>> mask_embed;

  CtPtr at(const CtPtr& a, int level) { return a->level == level ? a : level_align(cx, *a, level); }
  // at(xs[i], to[i]) for every i: alignments that share a source level, a
  // target level and a degree run as one batch, and a ciphertext listed
  // twice is aligned once
  std::vector<CtPtr> at_each(const std::vector<CtPtr>& xs, const std::vector<int>& to) {
    std::vector<CtPtr> out(xs.size());
    std::map<std::tuple<int, int, int>, std::vector<size_t>> groups;
    for (size_t i = 0; i < xs.size(); ++i) {
      if (xs[i]->level == to[i])
        out[i] = xs[i];
      else
        groups[{xs[i]->level, to[i], xs[i]->npoly}].push_back(i);
    }
    for (auto& g : groups) {
      std::vector<const Ciphertext*> src;
      std::map<const Ciphertext*, size_t> slot;
      for (size_t i : g.second)
        if (slot.emplace(xs[i].get(), src.size()).second) src.push_back(xs[i].get());
      const int level = std::get<1>(g.first);
      std::vector<CtPtr> r;
      if (src.size() == 1)
        r.push_back(level_align(cx, *src[0], level));
      else
        r = level_align_n(cx, src, level);
      for (size_t i : g.second) out[i] = r[slot[xs[i].get()]];
    }
    return out;
  }
  // x - mu for every x, at the lowest of their levels
  std::vector<CtPtr> sub_each(const std::vector<CtPtr>& X, const CtPtr& mu) {
    std::vector<CtPtr> ops(X);
    ops.push_back(mu);
    int m = mu->level;
    for (auto& x : X) m = std::min(m, x->level);
    auto al = at_each(ops, std::vector<int>(ops.size(), m));
    std::vector<CtPtr> out;
    for (size_t i = 0; i < X.size(); ++i) out.push_back(sub(cx, *al[i], *al.back()));
    return out;
  }
  CtPtr addx(const CtPtr& a, const CtPtr& b) {
    int m = std::min(a->level, b->level);
    return add(cx, *at(a, m), *at(b, m));
  }
  CtPtr subx(const CtPtr& a, const CtPtr& b) {
    int m = std::min(a->level, b->level);
    return sub(cx, *at(a, m), *at(b, m));
  }
  CtPtr mulx(const CtPtr& a, const CtPtr& b) {
    int m = std::min(a->level, b->level);
    return mul(cx, evk, *at(a, m), *at(b, m));
  }
  CtPtr sq(const CtPtr& a) { return mul(cx, evk, *a, *a); }
  // level_align results of one ciphertext, kept per level (T_1 is subtracted
  // from every odd Chebyshev term, several of which share a level)
  struct LevelCache {
    Circ* c;
    std::map<int, CtPtr> at_level;
    CtPtr get(const CtPtr& a, int level) {
      if (a->level == level) return a;
      auto it = at_level.find(level);
      if (it != at_level.end()) return it->second;
      return at_level[level] = c->at(a, level);
    }
  };
  // the InvSqrt argument mapped onto [-1, 1]; a pure shift (b - a = 2, Eq. 1's
  // x - 1 on [0, 2]) needs no product and no level
  CtPtr affine(const CtPtr& v, double a, double b) {
    const double g = 2.0 / (b - a);
    return add_const(cx, g == 1.0 ? *v : *mc(v, g), -(a + b) / (b - a));
  }
  // c a brought to `level` (below a's) with one rescale
  CtPtr lin1(const CtPtr& a, double c, int level) { return lincomb(cx, {a.get()}, {c}, level); }
  // sum_{k=1..d} c_k T_k with one rescale, one level below the lowest T_k
  CtPtr weighted(const std::vector<CtPtr>& T, const std::vector<double>& c, int d) {
    std::vector<const Ciphertext*> ts;
    std::vector<double> cs;
    int low = T[1]->level;
    for (int k = 1; k <= d; ++k) {
      ts.push_back(T[k].get());
      cs.push_back(c[k]);
      low = std::min(low, T[k]->level);
    }
    return lincomb(cx, ts, cs, low - 1);
  }
  CtPtr mc(const CtPtr& a, double c) { return mul_const(cx, *a, c); }
  // mc(x, c) of every x (one level): the rescales run batched
  std::vector<CtPtr> mc_n(const std::vector<CtPtr>& xs, double c) {
    if (xs.size() < 2) {
      std::vector<CtPtr> out;
      for (auto& x : xs) out.push_back(mc(x, c));
      return out;
    }
    std::vector<const Ciphertext*> p;
    for (auto& x : xs) p.push_back(x.get());
    return mul_const_n(cx, p, c);
  }
  CtPtr sum(const std::vector<CtPtr>& xs) {
    bool same = xs.size() > 2;
    for (auto& x : xs) same = same && x->level == xs[0]->level && x->scale == xs[0]->scale;
    if (same) {
      std::vector<const Ciphertext*> p;
      for (auto& x : xs) p.push_back(x.get());
      return add_n(cx, p);
    }
    CtPtr acc = xs[0];
    for (size_t i = 1; i < xs.size(); ++i) acc = addx(acc, xs[i]);
    return acc;
  }
  CtPtr rs(const CtPtr& a) {
    if (cx.router) return cx.router->rotsum(cx, evk, {a})[0];
    return rotsum(cx, evk, *a);
  }

  // RotSum(sum_c Z_c mask_c), mask 1/n on rows < n: the full ciphertexts are
  // added first and scaled by 1/n once; a ragged last one takes its row mask
  // Start encoding the row mask of an n-row column on a host thread (the
  // mask's values do not depend on the level; only the final rounding does)
  void prefetch_mask(size_t n) {
    const size_t S = (size_t)cx.P().slots(), rows = n % S;
    if (rows == 0) return;
    const Params* P = &cx.P();
    mask_rows = rows;
    mask_n = n;
    mask_embed = std::async(std::launch::async, [P, rows, n, S] {
                   std::vector<double> v(S, 0.0);
                   for (size_t j = 0; j < rows; ++j) v[j] = 1.0 / (double)n;
                   std::vector<long double> p;
                   encode_embed(*P, v.data(), (int)S, p);
                   return p;
                 }).share();
  }

  CtPtr mask_mean(const std::vector<CtPtr>& zs, size_t n) {
    const size_t S = (size_t)cx.P().slots();
    std::vector<CtPtr> full, terms;
    for (size_t c = 0; c < zs.size(); ++c) {
      size_t rows = std::min(S, n - c * S);
      if (rows == S) {
        full.push_back(zs[c]);
      } else {
        PtPtr pt;
        if (mask_embed.valid() && mask_rows == rows && mask_n == n) {
          pt = encode_embedded(cx, mask_embed.get(), zs[c]->level);
        } else {
          std::vector<double> v(S, 0.0);
          for (size_t j = 0; j < rows; ++j) v[j] = 1.0 / (double)n;
          pt = encode(cx, v.data(), S, zs[c]->level);
        }
        terms.push_back(mul_plain(cx, *zs[c], *pt));
      }
    }
    if (!full.empty()) terms.insert(terms.begin(), mc(sum(full), 1.0 / (double)n));
    return rs(sum(terms));
  }

  // Mean(x, B): the column's ciphertexts added, scaled by 1/(B n) once, summed
  CtPtr mean_B(const std::vector<CtPtr>& X, size_t n, double B) {
    return rs(mc(sum(X), 1.0 / (B * (double)n)));
  }

  CtPtr variance_B(const std::vector<CtPtr>& X, size_t n, double B, const CtPtr& mean_term) {
    auto xs = mc_n(X, 1.0 / (B * std::sqrt((double)n)));
    auto e2 = rs(sum(mulx_n(xs, xs)));
    auto m2 = sq(mean_term);
    return subx(e2, m2);
  }

  // Mean(x, B_mean) and Variance(x, B_var) with one two-lane RotSum: the
  // variance's slot sum does not need the mean, so the mean's sum is brought
  // to its level and both are summed together; Var = E2 - m^2 with
  // m = Mean(x, B_var)
  std::pair<CtPtr, CtPtr> moments(const std::vector<CtPtr>& X, size_t n, double B_mean,
                                  double B_var) {
    auto s1 = mc(sum(X), 1.0 / (B_mean * (double)n));
    auto xs = mc_n(X, 1.0 / (B_var * std::sqrt((double)n)));
    auto s2 = sum(mulx_n(xs, xs));
    auto r = rs_n({at(s1, s2->level), s2});
    CtPtr m = (B_var == B_mean) ? r[0] : mc(r[0], B_mean / B_var);
    return {r[0], subx(r[1], sq(m))};
  }

  std::vector<double> coeffs(const InvSqrtCfg& cfg, double Bp) {
    std::vector<double> base;
    if (!cfg.coeffs.empty()) {
      base = cfg.coeffs;
    } else {
      base = chebyshev_invsqrt(cfg.a, cfg.b, cfg.degree, 1.0);
    }
    const double r = std::sqrt(Bp);
    for (auto& v : base) v = v / r;
    return base;
  }

  // a refresh: down to level 0, then bootstrapped to the top computation level
  CtPtr refresh(const CtPtr& x, const Bootstrapper& bt) { return bootstrap(cx, evk, bt, *at(x, 0)); }

  std::pair<CtPtr, CtPtr> inv_sqrt(const CtPtr& v, double Bp, const InvSqrtCfg& cfg, int reserve = 0) {
    return inv_sqrt_n({v}, {Bp}, cfg, reserve)[0];
  }

  CtPtr sqrt_(const CtPtr& v, double Bp, const InvSqrtCfg& cfg, int reserve = 0) {
    auto yw = inv_sqrt(v, Bp, cfg, reserve);
    return mul_int(cx, *mulx(yw.second, yw.first), 2);
  }

  // u = x^2, w = u^2; terms 35/16 x, (-35/16 x) u, (21/16 x) w,
  // ((-5/16 x) u) w; the products of one level run as one batch
  CtPtr g3(const CtPtr& x) {
    auto u = sq(x);
    auto a1 = mc(x, 35.0 / 16.0);
    auto m3 = mc(x, -35.0 / 16.0), m5 = mc(x, 21.0 / 16.0), m7 = mc(x, -5.0 / 16.0);
    auto r = mulx_n({u, m3, m7}, {u, u, u});          // w, a3, (-5/16 x) u
    auto q = mulx_n({m5, r[2]}, {r[0], r[0]});        // a5, a7
    return sum({a1, r[1], q[0], q[1]});
  }

  // ---- the same sequences over several independent operands ("lanes"):
  // every lane performs exactly the operations of the one-operand helpers
  // above, and the products and RotSums of equal level run as one batch.
  std::vector<CtPtr> mulx_n(const std::vector<CtPtr>& a, const std::vector<CtPtr>& b) {
    std::vector<int> m(a.size());
    for (size_t i = 0; i < a.size(); ++i) m[i] = std::min(a[i]->level, b[i]->level);
    const std::vector<CtPtr> A = at_each(a, m), B = at_each(b, m);
    bool same = true;
    for (size_t i = 0; i < a.size(); ++i) same = same && A[i]->level == A[0]->level;
    if (!same || A.size() < 2) {
      std::vector<CtPtr> out;
      for (size_t i = 0; i < A.size(); ++i) out.push_back(mul(cx, evk, *A[i], *B[i]));
      return out;
    }
    std::vector<const Ciphertext*> pa, pb;
    for (size_t i = 0; i < A.size(); ++i) {
      pa.push_back(A[i].get());
      pb.push_back(B[i].get());
    }
    return mul_batch(cx, evk, pa, pb);
  }
  std::vector<CtPtr> rs_n(const std::vector<CtPtr>& xs) {
    bool same = true;
    for (auto& x : xs) same = same && x->level == xs[0]->level;
    if (same && xs.size() > 1)
      return cx.router ? cx.router->rotsum(cx, evk, xs) : rotsum_batch(cx, evk, xs);
    std::vector<CtPtr> out;
    for (auto& x : xs) out.push_back(rs(x));
    return out;
  }

  // sum_{k<=d} c[l][k] T_k(ts[l]) for every lane l: T_1 = t,
  // T_k = 2 T_m T_{m+1} - T_1 (k = 2m + 1) or 2 T_m^2 - 1 (k = 2m); the terms
  // with 2^w < k <= 2^(w+1) need only earlier ones and share a level, so
  // each such wave is one batch of products over all lanes; then c_1..c_d in
  // one weighted sum one level below the lowest T_k, and c_0 added
  std::vector<CtPtr> cheb_series_n(const std::vector<CtPtr>& ts,
                                   const std::vector<std::vector<double>>& c, int d) {
    const size_t nl = ts.size();
    if (d == 0) {   // a constant initial value: 0 t + c_0 (t's level, no product)
      std::vector<CtPtr> y(nl);
      for (size_t l = 0; l < nl; ++l) y[l] = add_const(cx, *mul_int(cx, *ts[l], 0), c[l][0]);
      return y;
    }
    std::vector<std::vector<CtPtr>> T(nl, std::vector<CtPtr>(d + 1));
    for (size_t l = 0; l < nl; ++l) T[l][1] = ts[l];
    std::vector<LevelCache> t1(nl, LevelCache{this});
    for (int w = 0; (1 << w) < d; ++w) {
      const int lo = (1 << w) + 1, hi = std::min(1 << (w + 1), d);
      std::vector<CtPtr> A, B;
      for (int k = lo; k <= hi; ++k)
        for (size_t l = 0; l < nl; ++l) {
          const int m = k / 2;
          A.push_back(T[l][m]);
          B.push_back(T[l][(k % 2) ? m + 1 : m]);
        }
      auto p = mulx_n(A, B);
      size_t i = 0;
      for (int k = lo; k <= hi; ++k)
        for (size_t l = 0; l < nl; ++l, ++i) {
          auto q = mul_int(cx, *p[i], 2);
          T[l][k] = (k % 2) ? subx(q, t1[l].get(T[l][1], q->level)) : add_const(cx, *q, -1.0);
        }
    }
    std::vector<CtPtr> y(nl);
    for (size_t l = 0; l < nl; ++l) {
      y[l] = add_const(cx, *weighted(T[l], c[l], d), c[l][0]);
      T[l].clear();
    }
    return y;
  }

  std::vector<std::pair<CtPtr, CtPtr>> inv_sqrt_n(const std::vector<CtPtr>& vs_in,
                                                  const std::vector<double>& Bps,
                                                  const InvSqrtCfg& cfg, int reserve = 0) {
    const double a = cfg.a, b = cfg.b;
    const int d = cfg.degree;
    const size_t nl = vs_in.size();
    const Bootstrapper* bt = cfg.boot;
    std::vector<CtPtr> vs(vs_in);
    if (bt) {
      // the affine map, the ladder (T_d lies ceil(log2 d) levels down) and
      // the weighted sum must fit above level 0
      int ladder = 0;
      while ((1 << ladder) < d) ++ladder;
      const int need = (2.0 / (b - a) == 1.0 ? 0 : 1) + (d >= 1 ? ladder + 1 : 0);
      for (size_t l = 0; l < nl; ++l)
        if (vs[l]->level < need) vs[l] = refresh(vs[l], *bt);
    }
    std::vector<std::vector<double>> c(nl);
    std::vector<CtPtr> ts(nl);
    for (size_t l = 0; l < nl; ++l) {
      c[l] = coeffs(cfg, Bps[l]);
      if ((int)c[l].size() != d + 1) PPST_THROW(ST_EINVAL, "coefficient table does not match the degree");
      ts[l] = affine(vs[l], a, b);
    }
    std::vector<CtPtr> y = cheb_series_n(ts, c, d), w2(nl);
    if (bt && d >= 1)   // Alg. 3: the Chebyshev initial value is bootstrapped
      for (size_t l = 0; l < nl; ++l) y[l] = refresh(y[l], *bt);
    for (size_t l = 0; l < nl; ++l) w2[l] = mc(vs[l], Bps[l] / 2.0);
    for (int it = 0; it < cfg.iters; ++it) {
      if (bt)   // a step takes two levels below min(level w2, level y)
        for (size_t l = 0; l < nl; ++l) {
          if (w2[l]->level < 2) w2[l] = refresh(w2[l], *bt);
          if (y[l]->level < 2) y[l] = refresh(y[l], *bt);
        }
      // y^2 and w2 y side by side, then their product
      std::vector<CtPtr> A(y), B(y);
      A.insert(A.end(), w2.begin(), w2.end());
      B.insert(B.end(), y.begin(), y.end());
      auto r = mulx_n(A, B);
      std::vector<CtPtr> y2(r.begin(), r.begin() + nl), p1(r.begin() + nl, r.end());
      auto p2 = mulx_n(p1, y2);
      for (size_t l = 0; l < nl; ++l) y[l] = subx(lin1(y[l], 1.5, p2[l]->level), p2[l]);
    }
    if (bt)
      for (size_t l = 0; l < nl; ++l)
        if (y[l]->level < reserve) y[l] = refresh(y[l], *bt);
    std::vector<std::pair<CtPtr, CtPtr>> out;
    for (size_t l = 0; l < nl; ++l) out.push_back({y[l], w2[l]});
    return out;
  }

  void check_depth(const std::vector<CtPtr>& X, int need) {
    for (auto& x : X)
      if (x->level < need)
        PPST_THROW(ST_ELEVEL, "statistic needs " + std::to_string(need) + " levels, input has " +
                               std::to_string(x->level));
  }
};

void check_column(const Params& P, const std::vector<CtPtr>& X, size_t nrows) {
  if (X.empty()) PPST_THROW(ST_EINVAL, "empty column");
  if (nrows == 0) PPST_THROW(ST_EINVAL, "row count is zero");
  size_t need = (nrows + P.slots() - 1) / P.slots();
  if (need != X.size())
    PPST_THROW(ST_EINVAL, "row count does not match the number of ciphertexts");
  for (auto& x : X)
    if (x->level != X[0]->level) PPST_THROW(ST_ESCALE, "column ciphertexts at different levels");
}

void check_cfg(const InvSqrtCfg& cfg) {
  if (!(cfg.a >= 0.0) || !(cfg.b > cfg.a)) PPST_THROW(ST_EDOMAIN, "InvSqrt interval needs 0 <= a < b");
  if (cfg.degree < 0 || cfg.degree > kMaxChebDegree)
    PPST_THROW(ST_EDOMAIN, "Chebyshev degree out of range");
  if (cfg.iters < 0 || cfg.iters > 32) PPST_THROW(ST_EDOMAIN, "Newton iteration count out of range");
}

// levels consumed by InvSqrt: affine map, ladder, coefficient products, Newton
int invsqrt_depth(const InvSqrtCfg& cfg) {
  int ladder = 0;
  while ((1 << ladder) < cfg.degree + 1) ++ladder;
  const int affine = 2.0 / (cfg.b - cfg.a) == 1.0 ? 0 : 1;
  return affine + (cfg.degree >= 1 ? ladder + 1 : 0) + 2 * cfg.iters;
}

}  // namespace

std::vector<double> chebyshev_invsqrt(double a, double b, int degree, double Bp) {
  const int n = degree + 1;
  std::vector<double> fx(n), th(n);
  const double pi = 3.14159265358979323846;
  for (int j = 0; j < n; ++j) {
    th[j] = pi * ((double)j + 0.5) / (double)n;
    double t = std::cos(th[j]);
    double v = a + (b - a) * (t + 1.0) / 2.0;
    fx[j] = 1.0 / std::sqrt(Bp * v);
  }
  std::vector<double> c(n);
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += fx[j] * std::cos((double)k * th[j]);
    c[k] = (k == 0 ? 1.0 : 2.0) * s / (double)n;
  }
  return c;
}

std::vector<CtPtr> cheb_series(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& ts,
                               const std::vector<double>& c) {
  if (ts.empty() || c.size() < 2) PPST_THROW(ST_EINVAL, "no lanes or no coefficients");
  Circ circ{cx, evk};
  const int d = (int)c.size() - 1;
  return circ.cheb_series_n(ts, std::vector<std::vector<double>>(ts.size(), c), d);
}

CtPtr stat_mean(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n, double B) {
  check_column(cx.P(), X, n);
  Circ c{cx, evk};
  c.check_depth(X, 1);
  return c.mean_B(X, n, B);
}

CtPtr stat_variance(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B) {
  check_column(cx.P(), X, n);
  Circ c{cx, evk};
  c.check_depth(X, 2);
  auto mu = c.mean_B(X, n, B);
  return c.variance_B(X, n, B, mu);
}

std::vector<CtPtr> stat_invsqrt(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X,
                                double B, const InvSqrtCfg& cfg) {
  if (X.empty()) PPST_THROW(ST_EINVAL, "no input ciphertexts");
  if (!(B > 0.0) || !std::isfinite(B)) PPST_THROW(ST_EDOMAIN, "B must be positive");
  for (auto& x : X)
    if (x->level != X[0]->level) PPST_THROW(ST_ESCALE, "input ciphertexts at different levels");
  check_cfg(cfg);
  Circ c{cx, evk};
  c.check_depth(X, 1 + (cfg.boot ? 0 : invsqrt_depth(cfg)));
  auto vs = c.mc_n(X, 1.0 / B);
  auto r = c.inv_sqrt_n(vs, std::vector<double>(X.size(), B), cfg);
  std::vector<CtPtr> out;
  for (auto& p : r) out.push_back(p.first);
  return out;
}

std::vector<CtPtr> stat_zscore(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X,
                               size_t n, double B, const InvSqrtCfg& cfg) {
  check_column(cx.P(), X, n);
  check_cfg(cfg);
  Circ c{cx, evk};
  c.check_depth(X, 4 + (cfg.boot ? 0 : invsqrt_depth(cfg)));
  auto mv = c.moments(X, n, B, B);
  auto mu = c.mc(mv.first, B);
  auto b = c.inv_sqrt(mv.second, B * B, cfg, 1).first;
  auto dx = c.sub_each(X, mu);
  return c.mulx_n(dx, std::vector<CtPtr>(dx.size(), b));
}

CtPtr stat_kurtosis(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B, const InvSqrtCfg& cfg, bool excess) {
  check_column(cx.P(), X, n);
  check_cfg(cfg);
  Circ c{cx, evk};
  c.check_depth(X, 6 + (cfg.boot ? 0 : invsqrt_depth(cfg)));
  c.prefetch_mask(n);
  auto mv = c.moments(X, n, B, B);
  auto var = mv.second;
  auto mu = c.mc(mv.first, B);
  auto x1 = c.sub_each(X, mu);
  auto x2 = c.mulx_n(x1, x1);
  auto num = c.mask_mean(c.mulx_n(x2, x2), n);
  auto i = c.inv_sqrt(var, B * B, cfg, 3).first;
  auto i2 = c.sq(i);
  // (num i^2) i^2 keeps every partial product near the result's size
  auto k = c.mulx(c.mulx(num, i2), i2);
  return excess ? add_const(cx, *k, -3.0) : k;
}

CtPtr stat_skewness(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B, const InvSqrtCfg& cfg) {
  check_column(cx.P(), X, n);
  check_cfg(cfg);
  Circ c{cx, evk};
  c.check_depth(X, 5 + (cfg.boot ? 0 : invsqrt_depth(cfg)));
  c.prefetch_mask(n);
  auto mv = c.moments(X, n, B, B);
  auto var = mv.second;
  auto mu = c.mc(mv.first, B);
  auto x1 = c.sub_each(X, mu);
  auto x2 = c.mulx_n(x1, x1);
  auto num = c.mask_mean(c.mulx_n(x2, x1), n);
  auto i = c.inv_sqrt(var, B * B, cfg, 2).first;
  auto i2 = c.sq(i);
  return c.mulx(c.mulx(num, i), i2);
}

CtPtr stat_cv(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
              double B_mean, double B_var, const InvSqrtCfg& cfg, int sign_k) {
  check_column(cx.P(), X, n);
  check_cfg(cfg);
  if (sign_k < 0 || sign_k > 8) PPST_THROW(ST_EDOMAIN, "sign composition count out of range");
  Circ c{cx, evk};
  const Bootstrapper* bt = cfg.boot;
  c.check_depth(X, bt ? 2 : 2 + 3 * sign_k + 1 + invsqrt_depth(cfg) + 3);
  auto mv = c.moments(X, n, B_mean, B_var);
  auto muB = mv.first;
  CtPtr sg = muB;
  // with a bootstrapper: the sign is refreshed before a g_3 step (depth 3)
  // that it lacks the levels for, and after the last one when it has fewer
  // than 3 (the product with mu and the final product); the inverse mean
  // and the standard deviation keep the 3 levels their products need
  for (int k = 0; k < sign_k; ++k) {
    if (bt && sg->level < 3) sg = c.refresh(sg, *bt);
    sg = c.g3(sg);
  }
  if (bt && sg->level < 3) sg = c.refresh(sg, *bt);
  auto ia = c.inv_sqrt(c.mulx(muB, sg), B_mean, cfg, 3).first;
  auto mu_inv = c.sq(ia);
  auto sigma = c.sqrt_(mv.second, B_var * B_var, cfg, 3);
  return c.mulx(c.mulx(sigma, mu_inv), sg);
}

CtPtr stat_pearson(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X,
                   const std::vector<CtPtr>& Y, size_t n, double Bx, double By,
                   const InvSqrtCfg& cfg) {
  check_column(cx.P(), X, n);
  check_column(cx.P(), Y, n);
  if (X.size() != Y.size() || X[0]->level != Y[0]->level)
    PPST_THROW(ST_EINVAL, "the two columns differ in length or level");
  check_cfg(cfg);
  Circ c{cx, evk};
  c.check_depth(X, 5 + (cfg.boot ? 0 : invsqrt_depth(cfg)));
  // Eq. 2's pre-scaled moments: Mean(x, B), E[x^2]/B^2 and E[xy]/(Bx By) are
  // five independent slot sums, summed together at one level (one batched
  // RotSum); Var_B = E2 - Mean^2, Cov_B = Exy - Mean(x) Mean(y) = Cov/(Bx By)
  const double nd = (double)n;
  auto xs = c.mc_n(X, 1.0 / (Bx * std::sqrt(nd)));
  auto ys = c.mc_n(Y, 1.0 / (By * std::sqrt(nd)));
  auto sx = c.mc(c.sum(X), 1.0 / (Bx * nd)), sy = c.mc(c.sum(Y), 1.0 / (By * nd));
  const size_t m = X.size();
  std::vector<CtPtr> lhs, rhs;
  for (size_t i = 0; i < m; ++i) { lhs.push_back(xs[i]); rhs.push_back(xs[i]); }
  for (size_t i = 0; i < m; ++i) { lhs.push_back(ys[i]); rhs.push_back(ys[i]); }
  for (size_t i = 0; i < m; ++i) { lhs.push_back(xs[i]); rhs.push_back(ys[i]); }
  auto pr = c.mulx_n(lhs, rhs);
  auto part = [&](size_t k) {
    return c.sum(std::vector<CtPtr>(pr.begin() + k * m, pr.begin() + (k + 1) * m));
  };
  auto sxx = part(0), syy = part(1), sxy = part(2);
  const int lv = sxx->level;
  auto r = c.rs_n({c.at(sx, lv), c.at(sy, lv), sxx, syy, sxy});
  auto mm = c.mulx_n({r[0], r[1], r[0]}, {r[0], r[1], r[1]});
  auto varx = c.subx(r[2], mm[0]);
  auto vary = c.subx(r[3], mm[1]);
  auto cov = c.subx(r[4], mm[2]);
  auto is = c.inv_sqrt_n({varx, vary}, {1.0, 1.0}, cfg, 2);
  return c.mulx(cov, c.mulx(is[0].first, is[1].first));
}

}  // namespace ppst

// boot.cpp -- CKKS bootstrapping: plan, plaintexts and the circuit.
#include "boot.h"

#include <cmath>
#include <thread>

#include "kern.h"
#include "stats.h"

namespace ppst {

namespace {

int ceil_log2(int x) {
  int b = 0;
  while ((1 << b) < x) ++b;
  return b;
}

// one level of a transform: layers 2^lo .. 2^hi, offsets in units of the
// smallest half-length u = 2^(lo-1); a group that reaches len = n has 2^g
// distinct offsets mod n (m in [0, 2^g)), any other 2^(g+1) - 1 (m in
// [-(2^g - 1), 2^g - 1]); b = 2^ceil(ceil(log2 R) / 2) baby steps
BootGroup make_group(int inverse, int lo, int hi, int logn, int level, int ckind) {
  BootGroup g;
  const int layers = hi - lo + 1;
  int R;
  if (hi == logn) {
    g.m0 = 0;
    R = 1 << layers;
  } else {
    g.m0 = -((1 << layers) - 1);
    R = (1 << (layers + 1)) - 1;
  }
  g.inverse = inverse;
  g.lo = lo;
  g.hi = hi;
  g.level = level;
  g.ckind = ckind;
  g.u = 1 << (lo - 1);
  g.b = 1 << ((ceil_log2(R) + 1) / 2);
  g.G = (R + g.b - 1) / g.b;
  return g;
}

long mod_n(long x, long n) {
  x %= n;
  return x < 0 ? x + n : x;
}

}  // namespace

BootPlan boot_plan(const Params& P) {
  if (!P.bootstrappable()) PPST_THROW(ST_EINVAL, "parameter set without bootstrapping levels");
  const int C = P.spec.boot_cts, E = P.spec.boot_evalmod, S = P.spec.boot_stc;
  BootPlan plan;
  if (C != S) PPST_THROW(ST_EINVAL, "CoeffToSlot and SlotToCoeff need as many levels");
  if (E != ceil_log2(plan.degree) + 1 + plan.r) PPST_THROW(ST_EINVAL, "EvalMod levels do not match its depth");
  const int logn = P.logN - 1;
  if (C > logn) PPST_THROW(ST_EINVAL, "more transform levels than layers");
  // layer ranges from len = n down, the larger groups on top
  std::vector<std::pair<int, int>> ranges;
  int hi = logn;
  for (int t = 0; t < C; ++t) {
    const int size = logn / C + (t < logn % C ? 1 : 0);
    ranges.push_back({hi - size + 1, hi});
    hi -= size;
  }
  for (int t = 0; t < C; ++t)
    plan.cts.push_back(make_group(1, ranges[t].first, ranges[t].second, logn, P.L - t, t == 0 ? 1 : 0));
  for (int t = 0; t < S; ++t) {
    const auto& rg = ranges[C - 1 - t];
    plan.stc.push_back(make_group(0, rg.first, rg.second, logn, P.Lc + S - t, 2));
  }
  return plan;
}

std::vector<long> boot_rotations(const Params& P) {
  const BootPlan plan = boot_plan(P);
  const long n = P.slots();
  std::vector<long> out;
  auto put = [&](long r) {
    r = mod_n(r, n);
    if (r && std::find(out.begin(), out.end(), r) == out.end()) out.push_back(r);
  };
  for (const auto* v : {&plan.cts, &plan.stc})
    for (const BootGroup& g : *v) {
      for (int i = 1; i < g.b; ++i) put((long)g.u * i);
      for (int j = 0; j < g.G; ++j) put((long)g.u * (g.m0 + (long)g.b * j));
    }
  std::sort(out.begin(), out.end());
  return out;
}

BootFactor boot_factor(const Params& P, const BootPlan& plan, const BootGroup& g) {
  BootFactor f;
  f.scale_out = P.scale[g.level - 1];
  f.scale_in = P.scale[g.level];
  f.q_l = P.q[g.level];
  f.scale_top = P.scale[P.L];
  f.q0 = P.q[0];
  f.scale0 = P.scale[0];
  f.K = plan.K;
  f.nsplit = P.spec.boot_stc;
  return f;
}

std::vector<double> evalmod_coeffs(int K, int r, int degree) {
  if (degree < 1 || K < 1 || r < 0) PPST_THROW(ST_EDOMAIN, "EvalMod degree, K and r out of range");
  const int n = degree + 1;
  const double pi = 3.14159265358979323846;
  std::vector<double> th(n), fx(n), c(n);
  for (int j = 0; j < n; ++j) {
    th[j] = pi * ((double)j + 0.5) / (double)n;
    fx[j] = std::cos(2.0 * pi * ((double)K * std::cos(th[j]) - 0.25) / std::ldexp(1.0, r));
  }
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += fx[j] * std::cos((double)k * th[j]);
    c[k] = (k == 0 ? 1.0 : 2.0) * s / (double)n;
  }
  return c;
}

std::unique_ptr<Bootstrapper> boot_create(Context& cx, const std::vector<double>& coeffs) {
  const Params& P = cx.P();
  auto bt = std::make_unique<Bootstrapper>();
  bt->plan = boot_plan(P);
  const BootPlan& plan = bt->plan;
  bt->coeffs = coeffs.empty() ? evalmod_coeffs(plan.K, plan.r, plan.degree) : coeffs;
  if ((int)bt->coeffs.size() != plan.degree + 1)
    PPST_THROW(ST_EINVAL, "EvalMod needs degree + 1 coefficients");
  const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  auto build = [&](const BootGroup& g) {
    BootLevel t;
    t.g = g;
    const size_t cells = (size_t)g.G * g.b;
    std::vector<int64_t> ints(cells * P.N);
    std::vector<uint8_t> used(cells);
    try {
      boot_group_coeffs(P.logN, g, boot_factor(P, plan, g), ints.data(), used.data(), threads);
    } catch (const std::runtime_error& e) {
      PPST_THROW(ST_EINVAL, e.what());
    }
    t.cells.resize(cells);
    for (size_t c = 0; c < cells; ++c)
      if (used[c]) t.cells[c] = plaintext_from_coeffs(cx, ints.data() + c * P.N, g.level, 1.0);
    return t;
  };
  for (const BootGroup& g : plan.cts) bt->cts.push_back(build(g));
  for (const BootGroup& g : plan.stc) bt->stc.push_back(build(g));
  std::vector<int64_t> e(P.N, 0);
  e[P.slots()] = -1;
  bt->neg_xn = plaintext_from_coeffs(cx, e.data(), P.L - P.spec.boot_cts, 1.0);
  e[P.slots()] = 1;
  bt->pos_xn = plaintext_from_coeffs(cx, e.data(), P.Lc + P.spec.boot_stc, 1.0);
  return bt;
}

CtPtr boot_lintrans(Context& cx, const EvalKeys& evk, const Ciphertext& a, const BootLevel& t) {
  const Params& P = cx.P();
  const BootGroup& g = t.g;
  const long n = P.slots();
  if (a.level != g.level) PPST_THROW(ST_ELEVEL, "transform level does not match the ciphertext's");
  std::vector<long> steps(g.b);
  for (int i = 0; i < g.b; ++i) steps[i] = mod_n((long)g.u * i, n);
  // baby steps: the rotations of a, their key switches sharing one ModUp
  const std::vector<CtPtr> baby = rotate_hoisted(cx, evk, a, steps);
  std::vector<const u64*> bp(g.b);
  for (int i = 0; i < g.b; ++i) bp[i] = baby[i]->buf.p;
  // inner sums of every giant step: one pass over the baby steps
  std::vector<CtPtr> inner(g.G);
  std::vector<const u64*> pts((size_t)g.G * g.b, nullptr);
  std::vector<u64*> outs(g.G, nullptr);
  for (int j = 0; j < g.G; ++j) {
    bool any = false;
    for (int i = 0; i < g.b; ++i) {
      const PtPtr& pt = t.cells[(size_t)j * g.b + i];
      if (pt) {
        pts[(size_t)j * g.b + i] = pt->buf.p;
        any = true;
      }
    }
    if (any) {
      inner[j] = new_ct(cx, a.level, a.scale);
      outs[j] = inner[j]->buf.p;
    }
  }
  const size_t per = (size_t)(a.level + 1) * P.N;
  k_bsgs_inner(*cx.sh, bp.data(), g.b, pts.data(), outs.data(), g.G, a.level + 1, per, per,
               cx.stream);
  // giant steps: each inner sum rotated into place, then one rescale
  std::vector<CtPtr> terms;
  for (int j = 0; j < g.G; ++j) {
    if (!inner[j]) continue;
    const long r = mod_n((long)g.u * (g.m0 + (long)g.b * j), n);
    terms.push_back(r ? rotate(cx, evk, *inner[j], r) : inner[j]);
  }
  std::vector<const Ciphertext*> tp;
  for (const CtPtr& x : terms) tp.push_back(x.get());
  CtPtr sum = tp.size() == 1 ? terms[0] : add_n(cx, tp);
  return rescale_as(cx, *sum, P.scale[a.level - 1]);
}

CtPtr coeff_to_slot(Context& cx, const EvalKeys& evk, const Bootstrapper& bt, const Ciphertext& a) {
  CtPtr w;
  const Ciphertext* x = &a;
  for (const BootLevel& t : bt.cts) {
    w = boot_lintrans(cx, evk, *x, t);
    x = w.get();
  }
  return w;
}

std::pair<CtPtr, CtPtr> boot_split(Context& cx, const EvalKeys& evk, const Bootstrapper& bt,
                                   const Ciphertext& w) {
  const Params& P = cx.P();
  if (w.level != bt.neg_xn->level) PPST_THROW(ST_ELEVEL, "split expects CoeffToSlot's output level");
  CtPtr cj = apply_galois(cx, evk, w, 2 * (u64)P.N - 1);
  CtPtr re = add(cx, w, *cj);
  CtPtr im = mul_plain_raw(cx, *sub(cx, w, *cj), *bt.neg_xn);
  return {re, im};
}

std::vector<CtPtr> eval_mod(Context& cx, const EvalKeys& evk, const Bootstrapper& bt,
                            const std::vector<CtPtr>& lanes) {
  std::vector<CtPtr> y = cheb_series(cx, evk, lanes, bt.coeffs);
  for (int it = 0; it < bt.plan.r; ++it) {
    std::vector<const Ciphertext*> a;
    for (const CtPtr& v : y) a.push_back(v.get());
    std::vector<CtPtr> sq = a.size() > 1 ? mul_batch(cx, evk, a, a)
                                         : std::vector<CtPtr>{mul(cx, evk, *a[0], *a[0])};
    for (size_t l = 0; l < y.size(); ++l) y[l] = add_const(cx, *mul_int(cx, *sq[l], 2), -1.0);
  }
  return y;
}

CtPtr slot_to_coeff(Context& cx, const EvalKeys& evk, const Bootstrapper& bt, const Ciphertext& re,
                    const Ciphertext& im) {
  if (im.level != bt.pos_xn->level) PPST_THROW(ST_ELEVEL, "SlotToCoeff expects EvalMod's output level");
  CtPtr w = add(cx, re, *mul_plain_raw(cx, im, *bt.pos_xn));
  for (const BootLevel& t : bt.stc) w = boot_lintrans(cx, evk, *w, t);
  return w;
}

CtPtr bootstrap(Context& cx, const EvalKeys& evk, const Bootstrapper& bt, const Ciphertext& a) {
  CtPtr w = coeff_to_slot(cx, evk, bt, *mod_raise(cx, a));
  bt.runs.fetch_add(1, std::memory_order_relaxed);
  auto ri = boot_split(cx, evk, bt, *w);
  w.reset();
  auto y = eval_mod(cx, evk, bt, {ri.first, ri.second});
  return slot_to_coeff(cx, evk, bt, *y[0], *y[1]);
}

}  // namespace ppst

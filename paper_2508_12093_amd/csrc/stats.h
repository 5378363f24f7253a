// stats.h -- encrypted statistics of PP-STAT (Sec. 5) over the evaluator.
#pragma once

#include "eval.h"

namespace ppst {

// Largest Chebyshev degree of the InvSqrt initial value (2^9 - 1, Sec. 5.1).
// The ladder keeps every T_k of a ciphertext until the weighted sum, so a
// degree-d initial value holds d + 1 ciphertexts per input at once.
constexpr int kMaxChebDegree = 511;

struct Bootstrapper;

struct InvSqrtCfg {
  double a = 1e-3, b = 1.0;    // interval of the Chebyshev initial value
  int degree = 7;              // Chebyshev degree
  int iters = 3;               // Newton iterations
  std::vector<double> coeffs;  // optional c_0..c_d of 1/sqrt(v) on [a, b] (B' = 1)
  // With a bootstrapper the chain's levels are refreshed inside InvSqrt
  // (each refresh: level_align to 0, then bootstrap): the argument when it
  // has fewer levels than the initial value's polynomial needs, the initial
  // value itself (Alg. 3), w2 or y before a Newton step that lacks its two
  // levels, and the result when fewer remain than the statistic needs after.
  const Bootstrapper* boot = nullptr;
};

// first-kind Chebyshev interpolation coefficients of 1/sqrt(Bp v) on [a, b]
// in t = (2 v - a - b) / (b - a)
std::vector<double> chebyshev_invsqrt(double a, double b, int degree, double Bp);

// sum_k c_k T_k(t) of each lane t (all of one level): the Chebyshev ladder
// of the InvSqrt initial value (T_2m = 2 T_m^2 - 1, T_2m+1 = 2 T_m T_m+1 - T_1,
// one weighted sum with one rescale, c_0 added), ceil(log2 d) + 1 levels
std::vector<CtPtr> cheb_series(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& ts,
                               const std::vector<double>& c);

CtPtr stat_mean(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n, double B);
CtPtr stat_variance(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B);
// CryptoInvSqrt slot by slot: InvSqrt(x / B; B) ~ 1/sqrt(x), one output per input
std::vector<CtPtr> stat_invsqrt(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X,
                                double B, const InvSqrtCfg& cfg);
std::vector<CtPtr> stat_zscore(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X,
                               size_t n, double B, const InvSqrtCfg& cfg);
CtPtr stat_kurtosis(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B, const InvSqrtCfg& cfg, bool excess);
CtPtr stat_skewness(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B, const InvSqrtCfg& cfg);
CtPtr stat_cv(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
              double B_mean, double B_var, const InvSqrtCfg& cfg, int sign_k);
CtPtr stat_pearson(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X,
                   const std::vector<CtPtr>& Y, size_t n, double Bx, double By,
                   const InvSqrtCfg& cfg);

}  // namespace ppst

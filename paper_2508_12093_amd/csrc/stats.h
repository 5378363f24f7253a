// stats.h -- encrypted statistics of PP-STAT (Sec. 5) over the evaluator.
#pragma once

#include "eval.h"

namespace ppst {

struct InvSqrtCfg {
  double a = 1e-3, b = 1.0;    // interval of the Chebyshev initial value
  int degree = 7;              // Chebyshev degree
  int iters = 3;               // Newton iterations
  std::vector<double> coeffs;  // optional c_0..c_d of 1/sqrt(v) on [a, b] (B' = 1)
};

// first-kind Chebyshev interpolation coefficients of 1/sqrt(Bp v) on [a, b]
// in t = (2 v - a - b) / (b - a)
std::vector<double> chebyshev_invsqrt(double a, double b, int degree, double Bp);

CtPtr stat_mean(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n, double B);
CtPtr stat_variance(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& X, size_t n,
                    double B);
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

// boot.h -- CKKS bootstrapping over the evaluator (the paper's Bootstrapping,
// Sec. 3.2 and Alg. 3, taken from the work it cites).
//
//   ModRaise     level 0 -> L: the plaintext becomes t = c + q_0 I
//   CoeffToSlot  BR U0^H / n, three levels of baby-step giant-step sums
//                (one rescale each), constant Delta_L / (2 K q_0) in the first:
//                slots (t_k + i t_{k+n}) / (2 K q_0), bit-reversed
//   split        re = w + conj w, im = -X^n (w - conj w): x / K, x = t_k / q_0
//   EvalMod      Chebyshev series of cos(2 pi (K u - 1/4) / 2^r), r double
//                angles: sin(2 pi x) = 2 pi c_k / q_0 up to a cubic term
//   SlotToCoeff  re + X^n im through U0 BR, three levels, constant
//                (q_0 / (2 pi Delta_0))^(1/3) each: the message at Delta_Lc
#pragma once

#include <atomic>

#include "boot_host.h"
#include "eval.h"

namespace ppst {

struct BootPlan {
  int K = 16;          // |t / q_0| < K
  int r = 4;           // double angles
  int degree = 27;     // Chebyshev degree (ladder depth 5, weighted sum 1)
  std::vector<BootGroup> cts, stc;
};

// the plan of a bootstrappable parameter set: log2(N/2) layers split in
// three (larger groups on the len = N/2 side), CoeffToSlot at levels L, L-1,
// L-2, SlotToCoeff at Lc+3, Lc+2, Lc+1
BootPlan boot_plan(const Params& P);
// every nonzero rotation step (mod N/2) the transforms use, ascending
std::vector<long> boot_rotations(const Params& P);
// the factor inputs of a group
BootFactor boot_factor(const Params& P, const BootPlan& plan, const BootGroup& g);
// first-kind Chebyshev interpolation of cos(2 pi (K u - 1/4) / 2^r) on [-1, 1]
std::vector<double> evalmod_coeffs(int K, int r, int degree);

struct BootLevel {
  BootGroup g;
  std::vector<PtPtr> cells;     // [G b], null where the group has no diagonal
};

struct Bootstrapper {
  BootPlan plan;
  std::vector<BootLevel> cts, stc;
  std::vector<double> coeffs;   // EvalMod's c_0..c_degree
  PtPtr neg_xn, pos_xn;         // -X^n at CoeffToSlot's output level, X^n at EvalMod's
  mutable std::atomic<u64> runs{0};   // bootstraps enqueued with this material
};

// the plaintexts of every group (host binary128 encoding, then the device's
// NTT); coeffs empty: evalmod_coeffs(K, r, degree)
std::unique_ptr<Bootstrapper> boot_create(Context& cx, const std::vector<double>& coeffs);

CtPtr boot_lintrans(Context& cx, const EvalKeys& evk, const Ciphertext& a, const BootLevel& t);
CtPtr coeff_to_slot(Context& cx, const EvalKeys& evk, const Bootstrapper& bt, const Ciphertext& a);
// (re, im) of CoeffToSlot's output
std::pair<CtPtr, CtPtr> boot_split(Context& cx, const EvalKeys& evk, const Bootstrapper& bt,
                                   const Ciphertext& w);
// EvalMod of each lane (all of one level), the lanes' products batched
std::vector<CtPtr> eval_mod(Context& cx, const EvalKeys& evk, const Bootstrapper& bt,
                            const std::vector<CtPtr>& lanes);
// SlotToCoeff of re + X^n im
CtPtr slot_to_coeff(Context& cx, const EvalKeys& evk, const Bootstrapper& bt, const Ciphertext& re,
                    const Ciphertext& im);
// the whole refresh: level 0 in, level Lc out
CtPtr bootstrap(Context& cx, const EvalKeys& evk, const Bootstrapper& bt, const Ciphertext& a);

}  // namespace ppst

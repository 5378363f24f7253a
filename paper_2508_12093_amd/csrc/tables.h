// tables.h -- device-resident CRT constant tables of key switching and rescale.
#pragma once

#include "core.h"

namespace ppst {

constexpr int kMaxAlpha = 16;     // limbs per key-switching digit
// primes below this bound run their NTT in FP64 (ntt.hip, FpArith), whose
// twiddle entries are then (double w, double w/q)
constexpr u64 kFpPrimeBound = 1ULL << 44;
constexpr int kMaxSpecial = 8;    // special primes

// ModDown table layout (one table serves every level); the rows of the first
// two blocks are padded with zeros to kMaxSpecial so that kernels can run
// their loops over special primes to a compile-time bound:
//   [kMaxSpecial][2]      (Phat_k^-1 mod p_k, Shoup companion), Phat_k = P / p_k
//   [L+1][kMaxSpecial]    Phat_k 2^64 mod q_i (Montgomery form: the kernels'
//                         sums over k come out of Acc30::redc as sum Phat_k ...;
//                         the K values of one q_i contiguous)
//   [L+1][2]              (P^-1 mod q_i, Shoup companion)
//   [nprimes]             h mod (prime), h = (P - 1) / 2, the rounding offset
//   [L+1][2]              (P mod q_i, Shoup companion)
//   [L+1][kMaxSpecial]    Phat_k P^-1 2^64 mod q_i (Montgomery form, for the
//                         fused ModDown + rescale: the sum comes out times P^-1)
//   [L+1]                 h P^-1 mod q_i
//   [kMaxSpecial]         h Phat_k^-1 mod p_k (the ModDown weights' offset: the
//                         inverse NTT before the conversion ends with
//                         N^-1 Phat_k^-1 on the special limbs, so a weight is
//                         its output plus this)
struct MdLayout {
  int K, L;
  __host__ __device__ MdLayout(int k, int l) : K(k), L(l) {}
  __host__ __device__ int phinv(int k) const { return 2 * k; }
  __host__ __device__ int phat(int k, int i) const { return 2 * kMaxSpecial + i * kMaxSpecial + k; }
  __host__ __device__ int pinv(int i) const { return 2 * kMaxSpecial + kMaxSpecial * (L + 1) + 2 * i; }
  __host__ __device__ int hmod(int p) const { return pinv(L + 1) + p; }
  __host__ __device__ int pmod(int i) const { return hmod(L + 1 + K) + 2 * i; }
  __host__ __device__ int phatp(int k, int i) const { return pmod(L + 1) + i * kMaxSpecial + k; }
  __host__ __device__ int hpinv(int i) const { return phatp(0, L + 1) + i; }
  __host__ __device__ int hphinv(int k) const { return hpinv(L + 1) + k; }
  __host__ __device__ int size() const { return hphinv(kMaxSpecial); }
};

// ModUp table of one level: for each digit j, [kMaxAlpha][2] (Qhat_i^-1 mod
// q_i, Shoup) for the digit's limbs i, then [ne][kMaxAlpha] Qhat_i 2^64 mod
// p(t) (Montgomery form, for Acc30::redc) for every extended limb t (one
// target's values contiguous); entries past the digit's limbs are zero.
__host__ __device__ inline size_t modup_digit_words(int ne) {
  return 2 * kMaxAlpha + (size_t)kMaxAlpha * ne;
}

// Build every table of a parameter set on the device (called once per Shared).
void build_tables(Shared& sh);

// ModUp table of a level: [beta][modup_digit_words(ne)]
const u64* modup_table(const Shared& sh, int level);
// final factors of the inverse transform whose output ModUp reads at a level:
// that output is then x_i Qhat_i^-1 mod q_i, the scaled digit ModUp sums
const u64* modup_ninv(const Shared& sh, int level);
// Rescale table for dropping q_level: [level][3] = (q_level^-1 mod q_i, Shoup, q_level mod q_i)
const u64* rescale_table(const Shared& sh, int level);

}  // namespace ppst

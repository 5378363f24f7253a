// dev.h -- device-side modular arithmetic and kernel argument structs.
#pragma once

#include "core.h"

namespace ppst {

// high 64 bits of a 64x64 product
__device__ __forceinline__ u64 mulhi(u64 a, u64 b) { return __umul64hi(a, b); }

// a * w mod q with the Shoup companion wp = floor(w 2^64 / q); result in [0, 2q)
__device__ __forceinline__ u64 mul_shoup_lazy(u64 a, u64 w, u64 wp, u64 q) {
  return a * w - mulhi(a, wp) * q;
}
__device__ __forceinline__ u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }
__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 wp, u64 q) {
  return csub(mul_shoup_lazy(a, w, wp, q), q);
}
__device__ __forceinline__ u64 addm(u64 a, u64 b, u64 q) { return csub(a + b, q); }
__device__ __forceinline__ u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// x = hi 2^64 + lo, x < 2^124, reduced mod q (q < 2^62) with R = floor(2^128/q):
// the quotient estimate hi(x R / 2^128) is at most 2 below floor(x/q).
__device__ __forceinline__ u64 reduce128(u64 hi, u64 lo, const Mod& m) {
  u64 t0 = mulhi(lo, m.r_lo);
  u64 p1_lo = lo * m.r_hi, p1_hi = mulhi(lo, m.r_hi);
  u64 p2_lo = hi * m.r_lo, p2_hi = mulhi(hi, m.r_lo);
  u64 s = t0 + p1_lo;
  u64 c = s < t0;
  u64 s2 = s + p2_lo;
  c += s2 < s;
  u64 quo = p1_hi + p2_hi + c + hi * m.r_hi;
  u64 r = lo - quo * m.q;
  r = csub(r, m.q);
  return csub(r, m.q);
}
__device__ __forceinline__ u64 mulm(u64 a, u64 b, const Mod& m) {
  return reduce128(mulhi(a, b), a * b, m);
}
// 128-bit accumulator
struct Acc {
  u64 hi = 0, lo = 0;
  __device__ __forceinline__ void mac(u64 a, u64 b) {
    u64 l = a * b;
    u64 h = mulhi(a, b);
    lo += l;
    hi += h + (lo < l);
  }
};
// Sum of products of residues below 2^60 in base 2^30: x = x1 2^30 + x0 and
// y = y1 2^30 + y0 with every half below 2^30, so each partial product is
// below 2^60 and a1 (two partials per term) holds 8 terms without overflow;
// a0 and a2 hold 16.  Each term costs four 32x32+64 multiply-adds and no
// carry handling.  Call fold() after every 8 terms to keep a1 in range.
constexpr uint32_t kMask30 = (1u << 30) - 1;
struct Split30 {
  uint32_t lo = 0, hi = 0;
  Split30() = default;
  __device__ __forceinline__ explicit Split30(u64 x)
      : lo((uint32_t)x & kMask30), hi((uint32_t)(x >> 30)) {}
};
struct Acc30 {
  u64 a0 = 0, a1 = 0, a2 = 0;
  __device__ __forceinline__ void mac(Split30 x, Split30 y) {
    a0 += (u64)x.lo * y.lo;
    a1 += (u64)x.lo * y.hi;
    a1 += (u64)x.hi * y.lo;
    a2 += (u64)x.hi * y.hi;
  }
  __device__ __forceinline__ void fold() {
    a1 += a0 >> 30;
    a0 &= kMask30;
    a2 += a1 >> 30;
    a1 &= kMask30;
  }
  // the sum a0 + a1 2^30 + a2 2^60 (below 2^124 for up to 16 terms) mod q
  __device__ __forceinline__ u64 reduce(const Mod& m) const {
    Acc30 f = *this;
    f.fold();    // disjoint fields: the 128-bit words without a carry chain
    return reduce128(f.a2 >> 4, f.a0 | (f.a1 << 30) | (f.a2 << 60), m);
  }
  // the sum times 2^-64 mod q (Montgomery's REDC), for sums below q 2^64:
  // at most 16 terms whose first factors are below 2^60 and whose second
  // factors (constants stored as c 2^64 mod q) are below q.  With
  // mm = lo (-q^-1) mod 2^64, x + mm q is a multiple of 2^64 whose low word
  // carries exactly when lo != 0, and (x + mm q) / 2^64 < 2q.
  // After a fold the fields a0, a1 < 2^30 and a2 no longer overlap, so the
  // 128-bit sum's words are plain shifts and ORs, with no carries.
  __device__ __forceinline__ u64 redc(const Mod& m) const {
    Acc30 f = *this;
    f.fold();
    const u64 lo = f.a0 | (f.a1 << 30) | (f.a2 << 60);
    const u64 hi = f.a2 >> 4;
    const u64 mm = lo * m.mneg;
    return csub(hi + mulhi(mm, m.q) + (lo != 0), m.q);
  }
};

// x < 2^64 reduced mod q by one Barrett step (floor(2^64/q) = r_hi)
__device__ __forceinline__ u64 reduce64(u64 x, const Mod& m) {
  u64 quo = mulhi(x, m.r_hi);
  u64 r = x - quo * m.q;
  r = csub(r, m.q);
  return csub(r, m.q);
}

// x < bound reduced mod q: one conditional subtraction where bound <= 2 q
// (the test is the same for every lane of a limb), else a Barrett step
__device__ __forceinline__ u64 reduce_below(u64 x, u64 bound, const Mod& m) {
  return bound <= 2 * m.q ? csub(x, m.q) : reduce64(x, m);
}

// a0 b1 + a1 b0 mod q (the tensor's middle term; below 2 q^2 < 2^124)
__device__ __forceinline__ u64 mul2_add(u64 a0, u64 b1, u64 a1, u64 b0, const Mod& m) {
  Acc acc;
  acc.mac(a0, b1);
  acc.mac(a1, b0);
  return reduce128(acc.hi, acc.lo, m);
}

// Automorphism X -> X^g in canonical NTT order: output slot j takes input
// slot j' with 2 brv(j') + 1 = (2 brv(j) + 1) g mod 2N.  g = 0 stands for the
// identity.  The map sends every aligned block of 2^s slots onto one aligned
// block (the low bits of 2 brv(j) + 1 come from the high bits of j), so
// permuted reads of a row stay inside one row.
__device__ __forceinline__ uint32_t galois_src(uint32_t j, uint32_t g, int logN) {
  if (g == 0) return j;
  const uint32_t e = 2 * (__brev(j) >> (32 - logN)) + 1;
  const uint32_t e2 = (e * g) & ((2u << logN) - 1);
  return __brev((e2 - 1) >> 1) >> (32 - logN);
}

// limb t -> combined prime index: t < nq ? t : pofs + (t - nq)
struct PrimeMap {
  int nq, pofs;
  __device__ __forceinline__ int operator()(int t) const { return t < nq ? t : pofs + (t - nq); }
};

}  // namespace ppst
